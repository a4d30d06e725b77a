// Device side of the masked plus.pair dot product C<M> = A plus.pair B^T:
// for every mask entry (i, j), C(i,j) = |A_i and B_j|.  Shared by the
// single-graph and the many-graph kernels.
//
// One wavefront owns a row i.  It marks A_i in private LDS: a bitmap over
// the ids below TC_BM_IDS and a small open-addressing table for larger
// ids (a row with too many large ids falls back to a binary search of A_i
// in memory).  The mask row is then taken 64 entries at a time: lane t
// fetches the bounds of B_j for the t-th entry, the rows are cut into
// 64-id units, and the wave walks the units in order, two at a time so
// that two coalesced loads are in flight, testing every id against the
// LDS sets.  In the triangle-count form (M = A = B = L, L strictly lower,
// rows sorted) the first entry of each row is skipped: L_j holds ids
// below j = L_i[0], which L_i does not.  After the descending-degree
// relabel almost every probed id is a high-degree vertex with a small id,
// so the bitmap answers nearly all probes with one LDS read.
#pragma once

#include "internal.h"

constexpr int TC_BLOCK = 256;
constexpr int TC_WAVES = TC_BLOCK / 64;
constexpr int TC_BM_IDS = 24576;              // ids covered by the LDS bitmap
constexpr int TC_BM_WORDS = TC_BM_IDS / 32;   // 3 KiB per wave
constexpr int TC_HS_LOG = 8;
constexpr int TC_HS_SLOTS = 1 << TC_HS_LOG;   // 1 KiB per wave
constexpr int TC_HS_MAX = TC_HS_SLOTS / 2;    // most large ids the table takes

struct TcArgs {
    int64_t nrows;
    const int64_t *Mrp;   // mask pattern: which (i, j) to compute
    const int32_t *Mci;
    const int64_t *Arp;   // rows tested for membership
    const int32_t *Aci;
    const int64_t *Brp;   // rows streamed
    const int32_t *Bci;
    int tc_form;          // M = A = B = L, strictly lower with sorted rows
    // Many graphs packed back to back: graph g owns rows [gbase[g],
    // gbase[g+1]) and its column ids are local, so row j of graph g is
    // row gbase[g] + j.  nullptr for a single matrix.
    const int64_t *gbase = nullptr;
    int64_t ngraphs = 0;
};

// Graph of packed row r (gbase ascending, ngraphs + 1 entries).
__device__ __forceinline__ int64_t tc_graph_of(const TcArgs &a, int64_t r)
{
    int64_t lo = 0, hi = a.ngraphs;   // last g with gbase[g] <= r
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.gbase[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

// A streamed segment of the flattened loop: the next segment's offset and
// the segment's start in Bci minus its own offset (32-bit form).
struct TcPair {
    uint32_t x, b;
};

struct TcWaveLds {
    union {
        int64_t seg_s[64];  // flattened streaming: segment starts
        TcPair seg_p[64];   // or, with 32-bit offsets, per streamed segment
                            // (next offset, start - offset)
    };
    uint32_t bm[TC_BM_WORDS + 1];   // word TC_BM_WORDS stays zero
    int32_t hs[TC_HS_SLOTS];
    int32_t seg_x[65];      // exclusive id offsets of the segments in seg_s
                            // (seg_x[cnt] = total)
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t bcast64(int64_t x, int src)
{
    const int lo = __shfl((int)(x & 0xffffffff), src, 64);
    const int hi = __shfl((int)(x >> 32), src, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ uint32_t tc_hash(int32_t x)
{
    return ((uint32_t)x * 0x9E3779B1u) >> (32 - TC_HS_LOG);
}

// Is k in A_i, for k >= TC_BM_IDS (past the LDS bitmap)?
__device__ __forceinline__ unsigned tc_member_large(const TcWaveLds &L, bool use_hash, const int32_t *Arow,
                                                    int64_t alen, int32_t k)
{
    if (use_hash) {
        uint32_t h = tc_hash(k);
        while (true) {
            const int32_t y = L.hs[h];
            if (y == k) return 1u;
            if (y < 0) return 0u;
            h = (h + 1) & (TC_HS_SLOTS - 1);
        }
    }
    int lo = 0, hi = (int)alen;   // (a row holds fewer than 2^31 ids)
    while (lo < hi) {
        const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
        if (Arow[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return (lo < (int)alen && Arow[lo] == k) ? 1u : 0u;
}

// Is k in A_i?
__device__ __forceinline__ unsigned tc_member(const TcWaveLds &L, bool use_hash, const int32_t *Arow,
                                              int64_t alen, int32_t k)
{
    // (the bit-field extract reads only the low 5 bits of its offset: k & 31)
    if (k < TC_BM_IDS) return __builtin_amdgcn_ubfe(L.bm[k >> 5], (unsigned)k, 1u);
    return tc_member_large(L, use_hash, Arow, alen, k);
}

// Mark the ids of Arow in the wave's LDS sets; returns whether the hash
// table holds the large ids (else membership of a large id is a binary
// search of Arow).  The trip count is the same for every lane, so each
// ballot sees the whole wave and the result is uniform.
__device__ __forceinline__ bool tc_mark(TcWaveLds &L, const int32_t *__restrict__ Arow, int64_t alen,
                                        unsigned lane, int32_t *first_id = nullptr)
{
    // (a row of L holds fewer than 2^31 ids: 32-bit positions)
    const int n = (int)alen;
    int nlarge = 0;
    if (first_id) *first_id = (int)lane < n ? Arow[lane] : -1;
#pragma unroll 4
    for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + (int)lane;
        const int32_t x = t < n ? Arow[t] : 0;
        if (t < n && x < TC_BM_IDS) atomicOr(&L.bm[x >> 5], 1u << (x & 31));
        nlarge += __popcll(__ballot(t < n && x >= TC_BM_IDS));
    }
    const bool use_hash = nlarge > 0 && nlarge <= TC_HS_MAX;
    if (use_hash) {
        for (int s = lane; s < TC_HS_SLOTS; s += 64) L.hs[s] = -1;
        wave_sync();
        for (int t = lane; t < n; t += 64) {
            const int32_t x = Arow[t];
            if (x >= TC_BM_IDS) {
                uint32_t h = tc_hash(x);
                while (atomicCAS(&L.hs[h], -1, x) != -1) h = (h + 1) & (TC_HS_SLOTS - 1);
            }
        }
    }
    wave_sync();
    return use_hash;
}

// Clear the bitmap words tc_mark set (the hash table is reset by the next
// tc_mark that uses it).
__device__ __forceinline__ void tc_unmark(TcWaveLds &L, const int32_t *__restrict__ Arow, int64_t alen,
                                          unsigned lane)
{
    wave_sync();
    for (int64_t t = lane; t < alen; t += 64) {
        const int32_t x = Arow[t];
        if (x < TC_BM_IDS) L.bm[x >> 5] = 0u;
    }
    wave_sync();
}

// tc_unmark without reading the row again: a row of at most 64 ids clears
// the words of the id each lane kept from tc_mark's first pass (first_id,
// -1 for none); a longer row clears the whole bitmap.
__device__ __forceinline__ void tc_unmark_kept(TcWaveLds &L, int32_t first_id, int64_t alen, unsigned lane)
{
    wave_sync();
    if (alen <= 64) {
        if (first_id >= 0 && first_id < TC_BM_IDS) L.bm[first_id >> 5] = 0u;
    } else {
        for (int x = lane; x < TC_BM_WORDS; x += 64) L.bm[x] = 0u;
    }
    wave_sync();
}

// Count, over up to 64 segments (lane t < cnt holds segment t: ids
// Bci[s, s+len)), the ids that are marked: unit u holds ids
// 64u .. 64u+63 of the concatenation, so short segments share units, and
// INFLIGHT units are loaded before any is probed.  Each lane finds
// the segment of its id by walking the wave's LDS copy of the segment
// offsets forward (its ids only increase), holding its current segment and
// the next offset in registers so that LDS is read only on a crossing.
// Unit loads in flight per wave: 7 for the single-graph count, 5 for the
// many-graph kernel, whose per-graph bookkeeping leaves fewer registers
// (each the faster of 5, 6 and 7 as measured at 2^20 and on a batch of
// 2,000 graphs of 2^8 to 2^16 vertices).
constexpr int TC_FLAT_INFLIGHT = 7;
constexpr int TC_FLAT_INFLIGHT_BATCHED = 5;

// With OFF32 every streamed id lies below 2^30 entries of Bci, so an id is
// loaded at a 32-bit byte offset from Bci (no 64-bit address arithmetic),
// and the segments of nonzero length (in lane order) go to L.seg_p as
// pairs: a crossing step reads the next offset and the start together.
// The other lanes below cnt keep s in L.seg_s after them, from slot
// nonzero-lengths-count on (a bitmap entry rides there to tc_bitmap_lanes).
template <int INFLIGHT = TC_FLAT_INFLIGHT, bool OFF32 = false>
__device__ __forceinline__ unsigned long long tc_stream_flat(TcWaveLds &L, bool use_hash,
                                                             const int32_t *__restrict__ Arow, int64_t alen,
                                                             const int32_t *__restrict__ Bci, int64_t s,
                                                             int len, int cnt, unsigned lane)
{
    const int incl = wave_incl_sum(len);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    if (OFF32) {
        const uint64_t mk = __ballot(len > 0);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
        if (len > 0) L.seg_p[below] = TcPair{(uint32_t)incl, (uint32_t)s - (uint32_t)(incl - len)};
        else if ((int)lane < cnt) L.seg_s[__popcll(mk) + (int)lane - below] = s;
    } else {
        if ((int)lane < cnt) {
            L.seg_s[lane] = s;
            L.seg_x[lane] = incl - len;
        }
        if (lane == 0) L.seg_x[cnt] = total;
    }
    wave_sync();
    unsigned acc = 0;   // (a lane probes one id in 64 of an int total)
    // the lane's current segment t (start s_t in Bci, offset x_t) and the
    // next one's offset nx, kept in registers: LDS is read only on a
    // crossing (px points at seg_x[t + 1], pp at seg_p[t]: a crossing step
    // is one pointer increment and one LDS read).
    // Id g of the concatenation is Bci[s_t - x_t + g]: cb holds s_t - x_t.
    const int32_t *px = &L.seg_x[1];
    const TcPair *pp = &L.seg_p[0];
    int nx;
    int64_t cb = 0;
    uint32_t cb32 = 0u;
    if (OFF32) {
        const TcPair p0 = *pp;
        nx = (int)p0.x;
        cb32 = p0.b;
    } else {
        nx = *px;
        cb = L.seg_s[0];
    }
    for (int g0 = 0; g0 < total; g0 += 64 * INFLIGHT) {
        int32_t k[INFLIGHT];
        bool v[INFLIGHT];
#pragma unroll
        for (int f = 0; f < INFLIGHT; f++) {
            const int g = g0 + 64 * f + (int)lane;
            v[f] = g < total;
            k[f] = -1;
            if (v[f]) {
                if (nx <= g) {
                    if (OFF32) {
                        TcPair pr;
                        do {
                            ++pp;
                            pr = *pp;
                        } while ((int)pr.x <= g);
                        nx = (int)pr.x;
                        cb32 = pr.b;
                    } else {
                        do {
                            ++px;
                            nx = *px;
                        } while (nx <= g);
                        const int t = (int)(px - &L.seg_x[1]);
                        cb = L.seg_s[t] - px[-1];
                    }
                }
                if (OFF32) k[f] = *(const int32_t *)((const char *)Bci + ((cb32 + (uint32_t)g) << 2));
                else k[f] = Bci[cb + g];
            }
        }
        // the bitmap probes of all units together (no branch: an id past
        // the bitmap, or a lane past the end with id -1, reads the zero
        // word after the bitmap), then the ids past the bitmap, in the
        // units that hold any
        uint32_t wd[INFLIGHT];
        bool large = false;
#pragma unroll
        for (int f = 0; f < INFLIGHT; f++) {
            const unsigned w = (unsigned)k[f] >> 5;
            wd[f] = L.bm[w < (unsigned)TC_BM_WORDS ? w : (unsigned)TC_BM_WORDS];
            large = large || k[f] >= TC_BM_IDS;
        }
#pragma unroll
        for (int f = 0; f < INFLIGHT; f++) acc += __builtin_amdgcn_ubfe(wd[f], (unsigned)k[f], 1u);
        if (__ballot(large)) {
#pragma unroll
            for (int f = 0; f < INFLIGHT; f++)
                if (__ballot(k[f] >= TC_BM_IDS))
                    acc += k[f] >= TC_BM_IDS ? tc_member_large(L, use_hash, Arow, alen, k[f]) : 0u;
        }
    }
    wave_sync();
    return (unsigned long long)acc;
}

// Row i by the whole wave.  Returns the row's total; with PER_ENTRY also
// writes entry_counts[q] for each mask entry q of the row.
template <bool PER_ENTRY>
__device__ unsigned long long tc_row(const TcArgs &a, int64_t i, TcWaveLds &L,
                                     int64_t *__restrict__ entry_counts, unsigned lane,
                                     int64_t bbase = 0)
{
    const int64_t a0 = a.Arp[i], alen = a.Arp[i + 1] - a0;
    const int64_t m0 = a.Mrp[i], mlen = a.Mrp[i + 1] - m0;
    const int32_t *Arow = a.Aci + a0;
    if (mlen == 0) return 0;
    if (alen == 0 || (a.tc_form && alen < 2)) {
        if (PER_ENTRY)
            for (int64_t t = lane; t < mlen; t += 64) entry_counts[m0 + t] = 0;
        return 0;
    }
    const bool use_hash = tc_mark(L, Arow, alen, lane);

    unsigned long long acc = 0;
    for (int64_t q0 = 0; q0 < mlen; q0 += 64) {
        const int nseg = (int)((mlen - q0) < 64 ? (mlen - q0) : 64);
        int64_t s = 0;
        int len = 0;
        if ((int)lane < nseg) {
            const int64_t q = q0 + lane;
            const int32_t j = a.Mci[m0 + q];
            s = a.Brp[bbase + j];
            len = (int)(a.Brp[bbase + j + 1] - s);
            if (a.tc_form && q == 0) len = 0;
        }
        // units of 64 ids: exclusive and inclusive unit offsets per segment
        const int nch = (len + 63) >> 6;
        const int incl = wave_incl_sum(nch);
        const int U = __builtin_amdgcn_readlane(incl, 63);
        const int excl = incl - nch;
        unsigned segcnt = 0;
        int t = 0;       // segment of the current unit (wave-uniform)
        int tend = __shfl(incl, 0, 64);
        for (int u = 0; u < U; u += 2) {
            // unit u
            while (u >= tend) {
                t++;
                tend = __shfl(incl, t, 64);
            }
            const int t1 = t;
            const int64_t base1 = bcast64(s, t1) + (int64_t)(u - __shfl(excl, t1, 64)) * 64;
            const int lim1 = __shfl(len, t1, 64) - (u - __shfl(excl, t1, 64)) * 64;
            // unit u + 1
            int t2 = t1, lim2 = 0;
            int64_t base2 = 0;
            if (u + 1 < U) {
                int tt = t1, te = tend;
                while (u + 1 >= te) {
                    tt++;
                    te = __shfl(incl, tt, 64);
                }
                t2 = tt;
                base2 = bcast64(s, t2) + (int64_t)(u + 1 - __shfl(excl, t2, 64)) * 64;
                lim2 = __shfl(len, t2, 64) - (u + 1 - __shfl(excl, t2, 64)) * 64;
            }
            const bool v1 = (int)lane < lim1, v2 = (int)lane < lim2;
            const int32_t k1 = v1 ? a.Bci[base1 + lane] : 0;
            const int32_t k2 = v2 ? a.Bci[base2 + lane] : 0;
            const unsigned h1 = v1 ? tc_member(L, use_hash, Arow, alen, k1) : 0u;
            const unsigned h2 = v2 ? tc_member(L, use_hash, Arow, alen, k2) : 0u;
            if (PER_ENTRY) {
                const unsigned c1 = __popcll(__ballot(h1 != 0));
                const unsigned c2 = __popcll(__ballot(h2 != 0));
                if ((int)lane == t1) segcnt += c1;
                if ((int)lane == t2) segcnt += c2;
            } else {
                acc += h1 + h2;
            }
        }
        if (PER_ENTRY && (int)lane < nseg) entry_counts[m0 + q0 + lane] = (int64_t)segcnt;
    }
    tc_unmark(L, Arow, alen, lane);
    return acc;
}

// Estimated cost of a row: the ids it streams plus a fixed charge for
// marking and clearing A_i.
constexpr int64_t TC_ROW_CHARGE = 64;

// First row r with prefix[r] >= target (prefix: n+1 ascending values).
__device__ __forceinline__ int64_t tc_lower_bound(const int64_t *prefix, int64_t n, int64_t target)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Wave `w` of `nw` takes the rows whose work prefix starts in its equal
// share [w*T/nw, (w+1)*T/nw) of the total T: a static partition balanced
// by the streamed ids, so a run of heavy rows is spread over many waves.
// With per_graph (packed graphs), each graph's total is added to
// per_graph[g]; the return value is then 0.
template <bool PER_ENTRY>
__device__ unsigned long long tc_rows_balanced(const TcArgs &a, TcWaveLds &L,
                                               int64_t *__restrict__ entry_counts,
                                               const int64_t *__restrict__ prefix, int64_t w,
                                               int64_t nw,
                                               unsigned long long *__restrict__ per_graph = nullptr)
{
    const unsigned lane = lane_id();
    for (int x = lane; x <= TC_BM_WORDS; x += 64) L.bm[x] = 0u;
    wave_sync();
    const int64_t T = prefix[a.nrows];
    const int64_t lo = (int64_t)((__int128)T * w / nw), hi = (int64_t)((__int128)T * (w + 1) / nw);
    const int64_t r0 = tc_lower_bound(prefix, a.nrows, lo);
    const int64_t r1 = tc_lower_bound(prefix, a.nrows, hi);
    unsigned long long acc = 0;
    if (!a.gbase) {
        for (int64_t r = r0; r < r1; r++)
            if (a.Mrp[r + 1] > a.Mrp[r]) acc += tc_row<PER_ENTRY>(a, r, L, entry_counts, lane);
        return acc;
    }
    if (r0 >= r1) return 0;
    // each lane holds a partial count: the flush sums the wave first (the
    // graph changes at the same row for every lane, so all lanes take part)
    auto flush = [&](int64_t gg) {
        unsigned long long t = acc;
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (t && lane == 0 && per_graph) atomicAdd(&per_graph[gg], t);
        acc = 0;
    };
    int64_t g = tc_graph_of(a, r0);
    int64_t gend = a.gbase[g + 1];
    for (int64_t r = r0; r < r1; r++) {
        while (r >= gend) {
            flush(g);
            g++;
            gend = a.gbase[g + 1];
        }
        if (a.Mrp[r + 1] > a.Mrp[r]) acc += tc_row<PER_ENTRY>(a, r, L, entry_counts, lane, a.gbase[g]);
    }
    flush(g);
    return 0;
}

// Work of each row (a fixed charge plus the ids it streams; 0 for an empty
// mask row), for the balanced partition.  Rows with at most 64 mask
// entries are summed by one lane, longer ones by the whole wave.
__device__ __forceinline__ void tc_row_work_wave(const TcArgs &a, int64_t r0, int64_t *work,
                                                 int64_t charge = TC_ROW_CHARGE)
{
    const unsigned lane = lane_id();
    const int64_t r = r0 + lane;
    int64_t m0 = 0, mlen = 0, base = 0;
    if (r < a.nrows) {
        m0 = a.Mrp[r];
        mlen = a.Mrp[r + 1] - m0;
        if (a.gbase) base = a.gbase[tc_graph_of(a, r)];
    }
    int64_t w = 0;
    if (mlen <= 64)
        for (int64_t q = (a.tc_form ? 1 : 0); q < mlen; q++) {
            const int64_t j = base + a.Mci[m0 + q];
            w += a.Brp[j + 1] - a.Brp[j];
        }
    uint64_t big = __ballot(mlen > 64);
    while (big) {
        const int t = __ffsll((unsigned long long)big) - 1;
        big &= big - 1;
        const int64_t bm0 = bcast64(m0, t), bl = bcast64(mlen, t), bb = bcast64(base, t);
        int64_t ww = 0;
        for (int64_t q = lane; q < bl; q += 64) {
            if (a.tc_form && q == 0) continue;
            const int64_t j = bb + a.Mci[bm0 + q];
            ww += a.Brp[j + 1] - a.Brp[j];
        }
        for (int o = 32; o > 0; o >>= 1) ww += __shfl_xor(ww, o, 64);
        if ((int)lane == t) w = ww;
    }
    if (r < a.nrows) work[r] = mlen > 0 ? w + charge : 0;
}

int tc_masked_dot(lagr_ctx ctx, const TcArgs &a, bool per_entry, unsigned long long *total_dev,
                  int64_t *entry_counts, char *msg);

// ------------------------------------------------- min-side count plan
//
// In the triangle-count form every pair (i, j) of L (j < i) contributes
// |L_i and L_j|, and both sets only hold ids below j: L_j entirely, L_i in
// its first p entries, where p is the position of j in row i.  The plan
// streams one of the two, about the shorter, and probes it against LDS
// marks of the other.  Virtual rows 0..n-1 ("A side", row i) mark L_i and
// stream whole rows L_j; virtual rows n..2n-1 ("B side", row j) mark L_j
// and stream the prefix L_i[0, p), for pairs whose L_j is more than twice
// as long as the prefix (hub columns by their own rule, in the plan
// builder).
// Pairs with p = 0 or an empty L_j contribute nothing and are dropped.  An
// entry packs the streamed segment as (offset << TC_PLAN_LEN_BITS) |
// length.  The virtual rows are cut into items of up to 64 entries; an
// item records its first entry and count and the row it marks.
//
// Bitmap pairs.  A B-side pair whose marked row j has a low id reads
// fewer words as bits than as ids when ceil(j/32) < p: L_i[0, p) is L_i
// below j, which the first ceil(j/32) words of a bitmap of L_i hold, and
// L_j's marks are a bitmap in LDS already, so the pair counts
// popcount(word & mark word) over those words instead of probing p ids
// (a row holding many of the highest-degree vertices pays for them once
// per hub pair otherwise; the bitmap form of a row in SuiteSparse's
// formats plays the same part).  Every row of L with such a pair keeps
// the bits of its ids below 32 * bw words in `bits` at boff(i), where bw
// covers its largest such j.  These pairs sit among row j's B entries as
// TC_PLAN_BITS | boff(i); a wave streams an item's segments and then reads
// the bitmaps of its flagged entries.
//
// Items are handed to waves a few at a time (tc_dyn_wave); consecutive
// items of a row usually go to the same wave, which then keeps the row's
// marks.
constexpr int TC_PLAN_LEN_BITS = 24;
constexpr int TC_PLAN_CNT_BITS = 7;
constexpr uint64_t TC_PLAN_BITS = 1ull << 63;   // bitmap entry flag
constexpr int TC_PLAN_WORDS_SHIFT = 40;          // an A pair's bitmap words (below: the offset)

// The pair (id j marked at position p of row i) is a bitmap pair.
__host__ __device__ __forceinline__ bool tc_bitmap_pair(int64_t j, int64_t p)
{
    return j < TC_BM_IDS && ((j + 31) >> 5) < p;
}

// Words of a whole row with largest id `last` and `len` ids, when an A pair
// streaming it does better reading them than the ids (and all lie below
// TC_BM_IDS, within the LDS marks); 0 otherwise.
__host__ __device__ __forceinline__ unsigned tc_full_words(int64_t last, int64_t len)
{
    const int64_t w = (last >> 5) + 1;
    return last < TC_BM_IDS && w < len ? (unsigned)w : 0u;
}

struct TcPlan {
    int64_t n = 0;          // rows of L
    int64_t nitems = 0;
    int64_t ent_cap = 0;    // entry slots, 2 nnz(L): every virtual row has its own region
    int64_t item_cap = 0;   // allocated items (>= nitems)
    int64_t *trp = nullptr;      // 2n+1: region starts of the virtual rows
    int64_t *irp = nullptr;      // 2n+1 item offsets of the virtual rows
    uint64_t *ent = nullptr;     // ent_cap packed segments; the tail of each region is unused
    uint64_t *item = nullptr;    // nitems: (first entry << TC_PLAN_CNT_BITS) | count
    int32_t *item_row = nullptr; // nitems: row of L the item marks
    int64_t nbits = 0;           // bitmap words in use (set once read back)
    int64_t bits_cap = 0;        // allocated bitmap words (nnz(L) bounds them)
    int64_t *boff = nullptr;     // n+1: bitmap word offsets of the rows of L
    unsigned long long *status = nullptr;   // 8 words: L's longest row, unsorted flag, -, items, nnz(L), words
    uint32_t *bits = nullptr;    // bitmaps of the rows with bitmap pairs
};

struct PlanArgs {
    int64_t nitems;
    const int64_t *nitems_dev = nullptr;   // when not null, the item count is read here
    const int64_t *Lrp;
    const int32_t *Lci;
    const uint64_t *ent;
    const uint64_t *item;
    const int32_t *item_row;
    const uint32_t *bits;
    // many packed graphs: the graph of each item and its counter (else null)
    const int32_t *item_graph = nullptr;
    unsigned long long *per_graph = nullptr;
};

// The plan's wave loop: each wave marks each item's row (again only when the
// row changes) and streams its segments.  Items are handed out dynamically:
// a static split by a cost model left waves busy for about 60% of the
// launch at 2^20 (the model misjudges some items), so each wave takes
// TC_DYN_ITEMS (or the caller's grain) consecutive items at a time from a
// counter.  There is one counter per XCD (ctr[TC_DYN_STRIDE * x], one
// cache line each), covering one contiguous eighth of the items, so the
// waves of an XCD keep working through neighbouring items (their streamed
// rows stay in that XCD's L2); a wave whose eighth is used up moves on to
// the next eighth in turn.  The counters must be zero at launch.  With
// BATCHED each graph's part of the count is added to per_graph[g] (the
// items of one graph are contiguous) and the result is 0.
constexpr int TC_BITS_INFLIGHT = 6;   // bitmap word loads in flight per lane

// The bitmap pairs of one item.  tc_stream_flat left the entries in
// L.seg_s[first .. cnt) (first: 0, or with OFF32 the number of segments of
// nonzero length, whose pairs fill the slots below); a bitmap entry is the
// plan's raw word (sign bit set: TC_PLAN_BITS), holding the bitmap offset
// of its streamed row and, for an A pair, the words to read (so no
// per-lane state has to live in registers across the streaming loop).  A
// B item's pairs all read the marked row's words: L_j's bits are in L.bm,
// all in its first mark_words words (they cover L_j's largest id, so
// mark_words <= ceil(j/32), which every streamed row's bitmap covers).  An
// A pair reads the whole of its streamed row L_j as bits (nwl words, all
// ids below TC_BM_IDS) against the marks of L_i.  The pairs are compacted
// into the segment slots of L and their (pair, word) grid is walked 64
// elements per load, TC_BITS_INFLIGHT loads in flight.  With one width nw,
// each lane steps its (pair, word) position forward by 64 elements per
// load (with 64-bit offsets the pair of element g is g / nw, by a multiply
// with ceil(2^32 / nw), exact while g * nw < 2^32: g < 64 * 768 here);
// with per-pair widths, each lane walks the pairs' word offsets forward as
// tc_stream_flat walks segments.
// With OFF32 every bitmap word lies below 2^30 words of bits (32-bit byte
// offsets from bits, as in tc_stream_flat).
template <bool OFF32 = false>
__device__ __forceinline__ unsigned long long tc_bitmap_lanes(TcWaveLds &L, const uint32_t *__restrict__ bits,
                                                              const int32_t *__restrict__ Arow, int64_t alen, int first,
                                                              int cnt, unsigned lane)
{
    const uint64_t x = first <= (int)lane && (int)lane < cnt ? (uint64_t)L.seg_s[lane] : 0ull;
    const bool flag = (x & TC_PLAN_BITS) != 0;
    const int64_t off = (int64_t)(x & ((1ull << TC_PLAN_WORDS_SHIFT) - 1));
    const int nwl = (int)((x & ~TC_PLAN_BITS) >> TC_PLAN_WORDS_SHIFT);
    wave_sync();
    const uint64_t M = __ballot(flag);
    const int np = __popcll(M);
    const int r = __popcll(M & ((1ull << lane) - 1));
    const bool varied = __ballot(flag && nwl > 0) != 0;   // an A item
    unsigned long long acc = 0;
    if (!varied) {
        const int nw = alen > 0 ? (Arow[alen - 1] >> 5) + 1 : 0;   // up to the marked row's largest id
        if (flag) L.seg_s[r] = off;
        wave_sync();
        const int total = np * nw;
        if (OFF32 && total > 0) {
            // element g = q nw + w: each lane steps its (pair q, word w)
            // forward by 64 elements per unit, so g < total is q < np; an
            // idle lane probes the zero word after the bitmap
            const int dq = 64 / nw, dw = 64 - dq * nw;
            int q = (int)lane / nw, w = (int)lane - q * nw;
            unsigned acc32 = 0;   // (at most 768 words of 32 bits per lane)
            for (int g0 = 0; g0 < total; g0 += 64 * TC_BITS_INFLIGHT) {
                int qf[TC_BITS_INFLIGHT], wf[TC_BITS_INFLIGHT];
                uint32_t base[TC_BITS_INFLIGHT], x[TC_BITS_INFLIGHT], y[TC_BITS_INFLIGHT];
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) {
                    qf[f] = q;
                    wf[f] = w;
                    w += dw;
                    q += dq;
                    if (w >= nw) {
                        w -= nw;
                        q++;
                    }
                }
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) base[f] = (uint32_t)L.seg_s[qf[f] < np ? qf[f] : 0];
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) {
                    const bool v = qf[f] < np;
                    x[f] = v ? *(const uint32_t *)((const char *)bits + ((base[f] + (uint32_t)wf[f]) << 2)) : 0u;
                    y[f] = L.bm[v ? wf[f] : TC_BM_WORDS];
                }
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) acc32 += (unsigned)__popc(x[f] & y[f]);
            }
            acc = acc32;
        } else if (!OFF32) {
            const unsigned long long magic = (0x100000000ull + (unsigned)nw - 1) / (unsigned)nw;   // 2^32 for nw = 1
            for (int g0 = 0; g0 < total; g0 += 64 * TC_BITS_INFLIGHT) {
                uint32_t x[TC_BITS_INFLIGHT], y[TC_BITS_INFLIGHT];
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) {
                    const int g = g0 + 64 * f + (int)lane;
                    const int q = (int)(((unsigned long long)(unsigned)g * magic) >> 32), w = g - q * nw;
                    const bool v = g < total;
                    x[f] = v ? bits[L.seg_s[q] + w] : 0u;
                    y[f] = v ? L.bm[w] : 0u;
                }
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) acc += (unsigned)__popc(x[f] & y[f]);
            }
        }
    } else {
        // exclusive word offsets of the flagged lanes, in lane order
        const int mine = flag ? nwl : 0;
        const int incl = wave_incl_sum(mine);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        if (OFF32) {
            // pairs (next offset, bits offset - offset) walked from registers
            // as tc_stream_flat walks its segments; cx: the current pair's
            // own offset
            if (flag) L.seg_p[r] = TcPair{(uint32_t)incl, (uint32_t)off - (uint32_t)(incl - mine)};
            wave_sync();
            const TcPair *pp = &L.seg_p[0];
            const TcPair p0 = *pp;
            int nx = (int)p0.x, cx = 0;
            uint32_t cb = p0.b;
            unsigned acc32 = 0;
            for (int g0 = 0; g0 < total; g0 += 64 * TC_BITS_INFLIGHT) {
                uint32_t x[TC_BITS_INFLIGHT], y[TC_BITS_INFLIGHT];
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) {
                    const int g = g0 + 64 * f + (int)lane;
                    x[f] = 0u;
                    y[f] = 0u;
                    if (g < total) {
                        if (nx <= g) {
                            TcPair pr;
                            do {
                                cx = nx;
                                ++pp;
                                pr = *pp;
                                nx = (int)pr.x;
                            } while (nx <= g);
                            cb = pr.b;
                        }
                        x[f] = *(const uint32_t *)((const char *)bits + ((cb + (uint32_t)g) << 2));
                        y[f] = L.bm[g - cx];
                    }
                }
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) acc32 += (unsigned)__popc(x[f] & y[f]);
            }
            acc = acc32;
        } else {
            if (flag) {
                L.seg_s[r] = off;
                L.seg_x[r] = incl - mine;
            }
            if (lane == 0) L.seg_x[np] = total;
            wave_sync();
            int t = 0;
            for (int g0 = 0; g0 < total; g0 += 64 * TC_BITS_INFLIGHT) {
                uint32_t x[TC_BITS_INFLIGHT], y[TC_BITS_INFLIGHT];
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) {
                    const int g = g0 + 64 * f + (int)lane;
                    x[f] = 0u;
                    y[f] = 0u;
                    if (g < total) {
                        while (L.seg_x[t + 1] <= g) t++;
                        const int w = g - L.seg_x[t];
                        x[f] = bits[L.seg_s[t] + w];
                        y[f] = L.bm[w];
                    }
                }
#pragma unroll
                for (int f = 0; f < TC_BITS_INFLIGHT; f++) acc += (unsigned)__popc(x[f] & y[f]);
            }
        }
    }
    wave_sync();
    return acc;
}

constexpr int64_t TC_DYN_ITEMS = 8;
constexpr int TC_DYN_STRIDE = 16;   // 128 bytes between counters
constexpr int TC_DYN_PARTS = 8;

template <bool BATCHED, bool OFF32 = false>
__device__ unsigned long long tc_dyn_wave(const PlanArgs &a, TcWaveLds &L, unsigned long long *ctr, int part,
                                          int64_t grain)
{
    const unsigned lane = lane_id();
    for (int x = lane; x <= TC_BM_WORDS; x += 64) L.bm[x] = 0u;
    wave_sync();
    const uint64_t lmask = (1ull << TC_PLAN_LEN_BITS) - 1;
    const int64_t N = a.nitems_dev ? *a.nitems_dev : a.nitems;
    unsigned long long acc = 0;
    int32_t marked = -1, first_id = -1, g = -1;
    int64_t alen = 0;
    const int32_t *Arow = nullptr;
    bool use_hash = false;
    auto flush = [&]() {
        unsigned long long t = acc;
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0 && t && g >= 0) atomicAdd(&a.per_graph[g], t);
        acc = 0;
    };
    for (int tries = 0; tries < TC_DYN_PARTS;) {
        const int p = (part + tries) % TC_DYN_PARTS;
        const int64_t r0 = N * p / TC_DYN_PARTS, r1 = N * (p + 1) / TC_DYN_PARTS;
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(&ctr[TC_DYN_STRIDE * p], 1ull);
        c = (unsigned long long)__shfl((long long)c, 0, 64);
        const int64_t k0 = r0 + (int64_t)c * grain;
        if (k0 >= r1) {
            tries++;
            continue;
        }
        const int64_t k1 = k0 + grain < r1 ? k0 + grain : r1;
        // the grabbed items' descriptors, up to 64 at a time, one per lane
        // (one load each), then read back item by item with readlane: an
        // item does not wait for its own descriptor load
        for (int64_t kc = k0; kc < k1; kc += 64) {
        const int kn = (int)(k1 - kc < 64 ? k1 - kc : 64);
        const bool hasl = (int)lane < kn;
        const uint64_t itv = hasl ? a.item[kc + lane] : 0ull;
        const int32_t mv = hasl ? a.item_row[kc + lane] : 0;
        const int32_t gv = (BATCHED && hasl) ? a.item_graph[kc + lane] : 0;
        auto item_at = [&](int q) {
            return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(itv >> 32), q) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)itv, q);
        };
        // each lane's entry of the next item is loaded while this one streams
        uint64_t xn = 0;
        {
            const uint64_t it0 = item_at(0);
            if ((int)lane < (int)(it0 & ((1u << TC_PLAN_CNT_BITS) - 1)))
                xn = a.ent[(int64_t)(it0 >> TC_PLAN_CNT_BITS) + lane];
        }
        for (int q = 0; q < kn; q++) {
            if (BATCHED) {
                const int32_t gk = __builtin_amdgcn_readlane(gv, q);
                if (gk != g) {
                    flush();
                    g = gk;
                }
            }
            const uint64_t it = item_at(q);
            const int32_t m = __builtin_amdgcn_readlane(mv, q);
            const int cnt = (int)(it & ((1u << TC_PLAN_CNT_BITS) - 1));
            const uint64_t xq = xn;
            xn = 0;
            if (q + 1 < kn) {
                const uint64_t itn = item_at(q + 1);
                if ((int)lane < (int)(itn & ((1u << TC_PLAN_CNT_BITS) - 1)))
                    xn = a.ent[(int64_t)(itn >> TC_PLAN_CNT_BITS) + lane];
            }
            int64_t s = 0;
            int len = 0;
            if ((int)lane < cnt) {
                const uint64_t x = xq;
                // a bitmap entry streams no ids: it rides in s, raw, to tc_bitmap_lanes
                const bool bitmap = (x & TC_PLAN_BITS) != 0;
                s = bitmap ? (int64_t)x : (int64_t)(x >> TC_PLAN_LEN_BITS);
                len = bitmap ? 0 : (int)(x & lmask);
            }
            const bool any_bitmap = __ballot(s < 0) != 0;
            const int nstream = OFF32 ? __popcll(__ballot(len > 0)) : 0;
            if (m != marked) {
                if (marked >= 0) tc_unmark_kept(L, first_id, alen, lane);
                Arow = a.Lci + a.Lrp[m];
                alen = a.Lrp[m + 1] - a.Lrp[m];
                use_hash = tc_mark(L, Arow, alen, lane, &first_id);
                marked = m;
            }
            acc += tc_stream_flat<BATCHED ? TC_FLAT_INFLIGHT_BATCHED : TC_FLAT_INFLIGHT, OFF32>(L, use_hash, Arow, alen,
                                                                                     a.Lci, s, len, cnt, lane);
            if (any_bitmap)
                acc += tc_bitmap_lanes<OFF32>(L, a.bits, Arow, alen, nstream, cnt, lane);
        }
        }
    }
    if (marked >= 0) tc_unmark_kept(L, first_id, alen, lane);
    if (BATCHED) {
        flush();
        return 0;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
}

