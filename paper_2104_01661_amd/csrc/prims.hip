// Device-wide primitives: exclusive scan, LSD radix sort, fills, CSR row
// offsets from sorted keys, row degrees.
#include "internal.h"

#include <atomic>
#include <chrono>

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Block-wide exclusive scan of one int64 per thread; returns the block total.
__device__ int64_t block_exclusive_scan(int64_t x, int64_t *lds_waves, int64_t &total)
{
    const unsigned lane = lane_id();
    const unsigned wave = threadIdx.x / warpSize;
    const unsigned nwaves = blockDim.x / warpSize;
    int64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(incl, d, 64);
        if ((int)lane >= d) incl += y;
    }
    if (lane == 63) lds_waves[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (unsigned w = 0; w < nwaves; w++) {
            int64_t t = lds_waves[w];
            lds_waves[w] = acc;
            acc += t;
        }
        lds_waves[nwaves] = acc;
    }
    __syncthreads();
    total = lds_waves[nwaves];
    int64_t excl = incl - x + lds_waves[wave];
    __syncthreads();
    return excl;
}

// A tile is SCAN_ITEMS rows of SCAN_BLOCK consecutive elements: thread t
// holds element t of each row (v[i] = element i * SCAN_BLOCK + t of the
// tile), so every load and store of a wave covers 64 consecutive elements.
// striped_scan sets excl[i] to the sum of the tile's elements before
// element (i, t) and returns the tile's total: each row is scanned across
// the block (within waves by shuffles, then over the wave totals in LDS),
// and row i starts after the totals of rows 0 .. i-1.
__device__ __forceinline__ int64_t striped_scan(const int64_t (&v)[SCAN_ITEMS], int64_t (&excl)[SCAN_ITEMS],
                                                int64_t (*wt)[SCAN_ITEMS])
{
    const unsigned lane = lane_id();
    const unsigned wave = threadIdx.x / 64;
    int64_t incl[SCAN_ITEMS];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) incl[i] = v[i];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; i++) {
            const int64_t y = __shfl_up(incl[i], d, 64);
            if ((int)lane >= d) incl[i] += y;
        }
    if (lane == 63)
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; i++) wt[wave][i] = incl[i];
    __syncthreads();
    int64_t row_start = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        int64_t before = 0, row = 0;
#pragma unroll
        for (int w = 0; w < SCAN_BLOCK / 64; w++) {
            const int64_t x = wt[w][i];
            before += (unsigned)w < wave ? x : 0;
            row += x;
        }
        excl[i] = row_start + before + incl[i] - v[i];
        row_start += row;
    }
    __syncthreads();   // wt is free again
    return row_start;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const int64_t *__restrict__ in,
                                                           int64_t *__restrict__ out, int64_t n,
                                                           int64_t *__restrict__ tile_sums)
{
    __shared__ int64_t wt[SCAN_BLOCK / 64][SCAN_ITEMS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    int64_t v[SCAN_ITEMS], excl[SCAN_ITEMS];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * SCAN_BLOCK;
        v[i] = idx < n ? in[idx] : 0;
    }
    const int64_t total = striped_scan(v, excl, wt);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * SCAN_BLOCK;
        if (idx < n) out[idx] = excl[i];
    }
    if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

// Two-pass form for up to SCAN_DIRECT tiles: k_tile_sums, then each block
// adds the sums of the tiles before it itself (at most SCAN_DIRECT values,
// from L2) and scans its tile, instead of scanning the sums in a third
// launch and adding them back in a fourth.
constexpr int64_t SCAN_DIRECT = 4096;

__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums(const int64_t *__restrict__ in, int64_t n,
                                                          int64_t *__restrict__ tile_sums)
{
    __shared__ int64_t lds[SCAN_BLOCK / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * SCAN_BLOCK;
        s += idx < n ? in[idx] : 0;
    }
    int64_t total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles_after(const int64_t *__restrict__ in,
                                                                 int64_t *__restrict__ out, int64_t n,
                                                                 const int64_t *__restrict__ tile_sums)
{
    __shared__ int64_t lds[SCAN_BLOCK / 64 + 1];
    __shared__ int64_t wt[SCAN_BLOCK / 64][SCAN_ITEMS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    int64_t v[SCAN_ITEMS], excl[SCAN_ITEMS];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * SCAN_BLOCK;
        v[i] = idx < n ? in[idx] : 0;
    }
    int64_t before = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += SCAN_BLOCK) before += tile_sums[t];
    int64_t prefix;
    block_exclusive_scan(before, lds, prefix);
    striped_scan(v, excl, wt);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * SCAN_BLOCK;
        if (idx < n) out[idx] = prefix + excl[i];
    }
}

__global__ void k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ tile_offs)
{
    const int64_t add = tile_offs[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int i = threadIdx.x; i < SCAN_TILE; i += blockDim.x) {
        int64_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

__global__ void k_total(const int64_t *__restrict__ in_last, const int64_t *__restrict__ out_last,
                        int64_t *__restrict__ dst)
{
    *dst = *in_last + *out_last;
}

}  // namespace

static int scan_level(lagr_ctx ctx, const int64_t *in, int64_t *out, int64_t n, int level,
                      char *msg)
{
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SCAN_BLOCK), 0, ctx->stream, in, out, n,
                           (int64_t *)nullptr);
        LAUNCH_CHECK();
        return LAGR_SUCCESS;
    }
    if (level >= 4) return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "scan: input too large");
    int64_t *sums = (int64_t *)ws_get(ctx, (WsSlot)(WS_SCAN_L0 + level), sizeof(int64_t) * tiles);
    if (!sums) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "scan workspace");
    if (tiles <= SCAN_DIRECT) {
        hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, n, sums);
        hipLaunchKernelGGL(k_scan_tiles_after, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, out, n,
                           sums);
        LAUNCH_CHECK();
        return LAGR_SUCCESS;
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, ctx->stream, in,
                       out, n, sums);
    LAUNCH_CHECK();
    TRY(scan_level(ctx, sums, sums, tiles, level + 1, msg));
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, ctx->stream, out, n,
                       sums);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

int scan_exclusive_i64(lagr_ctx ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                       char *msg)
{
    if (n <= 0) {
        if (total) *total = 0;
        return LAGR_SUCCESS;
    }
    int64_t last_in = 0;
    // the last input is needed after an in-place scan overwrote it
    if (total) TRY(stage_to_host(ctx, 8, in + n - 1, sizeof(int64_t), false, msg));
    TRY(scan_level(ctx, in, out, n, 0, msg));
    if (total) {
        TRY(stage_to_host(ctx, 16, out + n - 1, sizeof(int64_t), true, msg));
        last_in = ((int64_t *)ctx->pinned)[1];
        *total = last_in + ((int64_t *)ctx->pinned)[2];
    }
    return LAGR_SUCCESS;
}

// ------------------------------------------------------------ radix sort

namespace {

constexpr int RS_BLOCK = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ROUNDS;   // keys per block
constexpr int RS_WAVES = RS_BLOCK / 64;

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                      int shift, int64_t *__restrict__ hist,
                                                      int64_t nblocks)
{
    __shared__ unsigned cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; r++) {
        int64_t i = base + (int64_t)r * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: keys keep their order inside each digit.  Each round
// takes RS_BLOCK consecutive keys; inside a wave the lanes with an equal
// digit find each other with eight ballots.
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t *__restrict__ in,
                                                         uint64_t *__restrict__ out, int64_t n,
                                                         int shift,
                                                         const int64_t *__restrict__ offs,
                                                         int64_t nblocks)
{
    __shared__ int64_t run[256];
    __shared__ unsigned wcnt[RS_WAVES][256];
    __shared__ int64_t wbase[RS_WAVES][256];
    const unsigned lane = lane_id();
    const unsigned wave = threadIdx.x / 64;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RS_ROUNDS; r++) {
        for (int w = 0; w < RS_WAVES; w++) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * RS_BLOCK + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = valid ? in[i] : 0;
        unsigned digit = valid ? (unsigned)((key >> shift) & 255u) : 256u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bal = __ballot((digit >> b) & 1u);
            same &= ((digit >> b) & 1u) ? bal : ~bal;
        }
        const unsigned rank = __popcll(same & below);
        if (valid && rank == 0) wcnt[wave][digit] = __popcll(same);
        __syncthreads();
        {
            const unsigned d = threadIdx.x;
            int64_t acc = run[d];
            for (int w = 0; w < RS_WAVES; w++) {
                wbase[w][d] = acc;
                acc += wcnt[w][d];
            }
            run[d] = acc;
        }
        __syncthreads();
        if (valid) out[wbase[wave][digit] + rank] = key;
        __syncthreads();
    }
}

__global__ void k_copy_u64(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace

int radix_sort_u64(lagr_ctx ctx, uint64_t *keys, int64_t n, int nbits, char *msg)
{
    if (n <= 1 || nbits <= 0) return LAGR_SUCCESS;
    const int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
    uint64_t *tmp = (uint64_t *)ws_get(ctx, WS_SORT_TMP, sizeof(uint64_t) * n);
    int64_t *hist = (int64_t *)ws_get(ctx, WS_SORT_HIST, sizeof(int64_t) * 256 * nblocks);
    if (!tmp || !hist) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "radix sort workspace");
    uint64_t *src = keys, *dst = tmp;
    int passes = 0;
    for (int shift = 0; shift < nbits; shift += 8, passes++) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblocks), dim3(RS_BLOCK), 0, ctx->stream, src,
                           n, shift, hist, nblocks);
        LAUNCH_CHECK();
        TRY(scan_exclusive_i64(ctx, hist, hist, 256 * nblocks, nullptr, msg));
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblocks), dim3(RS_BLOCK), 0, ctx->stream,
                           src, dst, n, shift, hist, nblocks);
        LAUNCH_CHECK();
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != keys) {
        hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256, 65536)), dim3(256), 0, ctx->stream,
                           src, keys, n);
        LAUNCH_CHECK();
    }
    return LAGR_SUCCESS;
}

// ----------------------------------------------------------------- fills

namespace {
template <class T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
}  // namespace

int fill_i64(lagr_ctx ctx, int64_t *p, int64_t n, int64_t value, char *msg)
{
    if (n <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                       p, n, value);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

int fill_u32(lagr_ctx ctx, uint32_t *p, int64_t n, uint32_t value, char *msg)
{
    if (n <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                       p, n, value);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

int fill_u8(lagr_ctx ctx, uint8_t *p, int64_t n, uint8_t value, char *msg)
{
    if (n <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                       p, n, value);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

namespace {
// A few words device -> pinned host memory, stored at system scope and
// fenced; with a flag, thread 0 then stores seq to it with release order,
// so a host that sees seq there also sees the words.
__global__ void k_to_host(const uint32_t *__restrict__ src, uint32_t *dst, int64_t words, uint32_t *flag,
                          uint32_t seq)
{
    for (int64_t w = threadIdx.x; w < words; w += blockDim.x)
        __hip_atomic_store(dst + w, src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
    if (flag) {
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Wait for the flag store of sequence number seq.  The host polls the
// pinned word (a blocking stream sync sleeps until an interrupt, tens of
// microseconds after a short wait), asks the runtime every 64 polls whether
// the stream failed or drained, and after 2 ms of polling blocks instead.
int wait_host_flag(lagr_ctx ctx, uint32_t seq, char *msg)
{
    volatile uint32_t *f = (volatile uint32_t *)((char *)ctx->pinned + LAGR_PINNED_SEQ);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; it++) {
        if (*f == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            flush_deferred(ctx);        // the stream has run up to the flag
            return LAGR_SUCCESS;
        }
        if ((it & 63u) == 0) {
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady)
                return lagr_fail(msg, LAGR_DEVICE_ERROR, "stream: %s", hipGetErrorString(e));
            if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (*f != seq) return lagr_fail(msg, LAGR_DEVICE_ERROR, "host flag %u not set after the stream drained", seq);
    std::atomic_thread_fence(std::memory_order_acquire);
    flush_deferred(ctx);
    return LAGR_SUCCESS;
}
}  // namespace

int stage_to_host(lagr_ctx ctx, size_t offset, const void *dev, size_t bytes, bool wait, char *msg)
{
    if (offset > LAGR_PINNED_STAGE || bytes > LAGR_PINNED_STAGE - offset)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "stage_to_host: %zu bytes at %zu exceed the staging buffer",
                         bytes, offset);
    const bool words = ((uintptr_t)dev & 3u) == 0 && (bytes & 3u) == 0 && (offset & 3u) == 0;
    if (!words) {
        HIP_TRY(hipMemcpyAsync((char *)ctx->pinned + offset, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
        if (wait) {
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            flush_deferred(ctx);
        }
        return LAGR_SUCCESS;
    }
    if (bytes == 0 && !wait) return LAGR_SUCCESS;
    const uint32_t seq = ++ctx->host_seq;
    hipLaunchKernelGGL(k_to_host, dim3(1), dim3(64), 0, ctx->stream, (const uint32_t *)dev,
                       (uint32_t *)((char *)ctx->pinned_dev + offset), (int64_t)(bytes / 4),
                       wait ? (uint32_t *)((char *)ctx->pinned_dev + LAGR_PINNED_SEQ) : nullptr, seq);
    HIP_TRY(hipGetLastError());
    return wait ? wait_host_flag(ctx, seq, msg) : LAGR_SUCCESS;
}

int host_wait(lagr_ctx ctx, char *msg)
{
    return stage_to_host(ctx, 0, ctx->pinned_dev, 0, true, msg);
}

int read_back(lagr_ctx ctx, void *host, const void *dev, size_t bytes, char *msg)
{
    if (bytes > LAGR_PINNED_STAGE) return lagr_fail(msg, LAGR_INVALID_VALUE, "read_back: too large");
    TRY(stage_to_host(ctx, 0, dev, bytes, true, msg));
    memcpy(host, ctx->pinned, bytes);
    return LAGR_SUCCESS;
}

// ------------------------------------------------ CSR offsets from keys

namespace {
// rowptr[r] = first position whose row >= r (a lower bound per row).
__global__ void k_rowptr_from_keys(const uint64_t *__restrict__ keys, int64_t nnz, int shift,
                                   int64_t nrows, int64_t *__restrict__ rowptr)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(keys[mid] >> shift) < r) lo = mid + 1;
            else hi = mid;
        }
        rowptr[r] = lo;
    }
}

// deg[v], the largest degree into m[0] and the number of degrees above
// big into m[1] (both zero on entry)
__global__ void k_degrees(const int64_t *__restrict__ rowptr, int64_t n, int64_t *__restrict__ deg, int64_t big,
                          unsigned long long *__restrict__ m)
{
    int64_t local = 0;
    unsigned long long nbig = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = rowptr[v + 1] - rowptr[v];
        deg[v] = d;
        local = d > local ? d : local;
        nbig += d > big ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        int64_t y = __shfl_xor(local, o, 64);
        local = y > local ? y : local;
        nbig += __shfl_xor(nbig, o, 64);
    }
    // one atomic per workgroup (atomics on one address serialise)
    __shared__ unsigned long long wmax, wbig;
    if (threadIdx.x == 0) wmax = wbig = 0;
    __syncthreads();
    if (lane_id() == 0) {
        atomicMax(&wmax, (unsigned long long)local);
        if (nbig) atomicAdd(&wbig, nbig);
    }
    __syncthreads();
    if (threadIdx.x == 0 && wmax) atomicMax(m, wmax);
    if (threadIdx.x == 0 && wbig) atomicAdd(m + 1, wbig);
}
}  // namespace

int rowptr_from_sorted_keys(lagr_ctx ctx, const uint64_t *keys, int64_t nnz, int shift,
                            int64_t nrows, int64_t *rowptr, char *msg)
{
    hipLaunchKernelGGL(k_rowptr_from_keys, dim3(grid_for(nrows + 1, 256, 65536)), dim3(256), 0,
                       ctx->stream, keys, nnz, shift, nrows, rowptr);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

namespace {
__global__ void k_chunk_counts(const int64_t *__restrict__ rp, int64_t n, int64_t min_len,
                               int64_t chunk, int64_t *__restrict__ cnt)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t len = rp[r + 1] - rp[r];
        cnt[r] = len > min_len ? (len + chunk - 1) / chunk : 0;
    }
}

__global__ void k_chunk_fill(const int64_t *__restrict__ rp, int64_t n, int64_t min_len, int64_t chunk,
                             const int64_t *__restrict__ off, int32_t *__restrict__ row,
                             int64_t *__restrict__ beg, int64_t *__restrict__ end)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rp[r], e = rp[r + 1];
        if (e - b <= min_len) continue;
        int64_t o = off[r];
        for (int64_t s = b; s < e; s += chunk, o++) {
            row[o] = (int32_t)r;
            beg[o] = s;
            end[o] = s + chunk < e ? s + chunk : e;
        }
    }
}
}  // namespace

int row_chunks(lagr_ctx ctx, const int64_t *rowptr, int64_t nrows, int64_t min_len, int64_t chunk,
               WsSlot count_slot, WsSlot list_slot, RowChunks *out, char *msg)
{
    out->n = 0;
    int64_t *cnt = (int64_t *)ws_get(ctx, count_slot, sizeof(int64_t) * (nrows + 1));
    if (!cnt) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "chunk workspace");
    if (nrows <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_chunk_counts, dim3(grid_for(nrows, 256, 16384)), dim3(256), 0, ctx->stream,
                       rowptr, nrows, min_len, chunk, cnt);
    LAUNCH_CHECK();
    int64_t total = 0;
    TRY(scan_exclusive_i64(ctx, cnt, cnt, nrows, &total, msg));
    if (total == 0) return LAGR_SUCCESS;
    char *lst = (char *)ws_get(ctx, list_slot, (size_t)total * 24 + 64);
    if (!lst) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "chunk list");
    int64_t *beg = (int64_t *)lst;
    int64_t *end = beg + total;
    int32_t *row = (int32_t *)(end + total);
    hipLaunchKernelGGL(k_chunk_fill, dim3(grid_for(nrows, 256, 16384)), dim3(256), 0, ctx->stream,
                       rowptr, nrows, min_len, chunk, cnt, row, beg, end);
    LAUNCH_CHECK();
    out->n = total;
    out->row = row;
    out->beg = beg;
    out->end = end;
    return LAGR_SUCCESS;
}

int row_degrees(lagr_ctx ctx, const int64_t *rowptr, int64_t n, int64_t *deg, int64_t *maxdeg,
                char *msg, int64_t big, int64_t *nbig)
{
    unsigned long long *m = (unsigned long long *)ws_get(ctx, WS_COUNTERS, 64);
    if (!m) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "counters");
    TRY(fill_i64(ctx, (int64_t *)m, 2, 0, msg));
    if (n > 0) {
        hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, 256)), dim3(256), 0, ctx->stream,
                           rowptr, n, deg, big, m);
        LAUNCH_CHECK();
    }
    unsigned long long h[2] = {0, 0};
    TRY(read_back(ctx, h, m, sizeof(h), msg));
    if (maxdeg) *maxdeg = (int64_t)h[0];
    if (nbig) *nbig = (int64_t)h[1];
    return LAGR_SUCCESS;
}
