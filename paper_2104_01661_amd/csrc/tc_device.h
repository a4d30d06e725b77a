// Device side of the masked plus.pair dot product: one wavefront per row,
// A_i hashed into LDS, the rows B_j of the mask row streamed as one
// flattened, load-balanced sequence.  Shared by the single-graph and the
// many-graph kernels.
#pragma once

#include "internal.h"

constexpr int TC_BLOCK = 256;
constexpr int TC_WAVES = TC_BLOCK / 64;
constexpr int TC_HASH_LOG = 11;
constexpr int TC_HASH_CAP = 1 << TC_HASH_LOG;    // int32 slots per wave
constexpr int TC_HASH_MAX_ROW = TC_HASH_CAP / 2;  // longest A_i the table takes

struct TcArgs {
    int64_t nrows;
    const int64_t *Mrp;   // mask pattern: which (i, j) to compute
    const int32_t *Mci;
    const int64_t *Arp;   // hashed rows
    const int32_t *Aci;
    const int64_t *Brp;   // streamed rows
    const int32_t *Bci;
    int skip_short;       // M = A = B = L: rows with < 2 entries count nothing
};

struct TcWaveLds {
    int32_t hash[TC_HASH_CAP];
    int64_t off[64];      // exclusive offsets of the chunk's segments
    int64_t start[64];    // where each segment starts in Bci
    uint32_t cnt[64];     // per-segment counts (per-entry output)
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t tc_hash(int32_t x, int shift)
{
    return ((uint32_t)x * 0x9E3779B1u) >> shift;
}

// Count |A_i and B_j| for the mask entries of row i.  Returns the row's
// total; with PER_ENTRY also writes entry_counts[q] for each mask entry q.
template <bool PER_ENTRY>
__device__ unsigned long long tc_row(const TcArgs &a, int64_t i, TcWaveLds &L,
                                     int64_t *__restrict__ entry_counts)
{
    const unsigned lane = lane_id();
    const int64_t a0 = a.Arp[i], alen = a.Arp[i + 1] - a0;
    const int64_t m0 = a.Mrp[i], mlen = a.Mrp[i + 1] - m0;
    if (mlen == 0) return 0;
    if (alen > TC_HASH_MAX_ROW) return 0;   // the big-row kernel takes it
    if (alen == 0 || (a.skip_short && alen < 2)) {
        if (PER_ENTRY)
            for (int64_t t = lane; t < mlen; t += 64) entry_counts[m0 + t] = 0;
        return 0;
    }
    int logc = 6;
    while ((int64_t(1) << logc) < 2 * alen) logc++;
    const uint32_t cap = 1u << logc, mask = cap - 1;
    const int shift = 32 - logc;
    for (uint32_t s = lane; s < cap; s += 64) L.hash[s] = -1;
    wave_sync();
    for (int64_t t = lane; t < alen; t += 64) {
        const int32_t x = a.Aci[a0 + t];
        uint32_t h = tc_hash(x, shift);
        while (atomicCAS(&L.hash[h], -1, x) != -1) h = (h + 1) & mask;
    }
    wave_sync();
    unsigned long long acc = 0;
    for (int64_t t0 = 0; t0 < mlen; t0 += 64) {
        const int nseg = (int)((mlen - t0) < 64 ? (mlen - t0) : 64);
        int64_t wl = 0, st = 0;
        if ((int)lane < nseg) {
            const int32_t j = a.Mci[m0 + t0 + lane];
            st = a.Brp[j];
            wl = a.Brp[j + 1] - st;
        }
        int64_t incl = wl;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(incl, d, 64);
            if ((int)lane >= d) incl += y;
        }
        L.off[lane] = incl - wl;
        L.start[lane] = st;
        if (PER_ENTRY) L.cnt[lane] = 0;
        const int64_t tot = __shfl(incl, 63, 64);
        wave_sync();
        for (int64_t p = lane; p < tot; p += 64) {
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.off[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            const int32_t k = a.Bci[L.start[lo] + (p - L.off[lo])];
            uint32_t h = tc_hash(k, shift);
            bool hit = false;
            while (true) {
                const int32_t y = L.hash[h];
                if (y == k) {
                    hit = true;
                    break;
                }
                if (y == -1) break;
                h = (h + 1) & mask;
            }
            if (hit) {
                if (PER_ENTRY) atomicAdd(&L.cnt[lo], 1u);
                else acc++;
            }
        }
        wave_sync();
        if (PER_ENTRY) {
            if ((int)lane < nseg) entry_counts[m0 + t0 + lane] = (int64_t)L.cnt[lane];
            wave_sync();
        }
    }
    return acc;
}

int tc_masked_dot(lagr_ctx ctx, const TcArgs &a, int64_t max_arow, bool per_entry,
                  unsigned long long *total_dev, int64_t *entry_counts, char *msg);
