// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/lagr.h"

#include <string>
#include <utility>
#include <vector>

// ------------------------------------------------------------------ errors

int lagr_fail(char *msg, int code, const char *fmt, ...);
static inline int lagr_ok(char *msg)
{
    if (msg) msg[0] = '\0';
    return LAGR_SUCCESS;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "%s failed: %s", #expr,            \
                             hipGetErrorString(e_));                                    \
    } while (0)

#define LAUNCH_CHECK()                                                                  \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return lagr_fail(msg, LAGR_DEVICE_ERROR, "kernel launch failed at %s:%d: %s",\
                             __FILE__, __LINE__, hipGetErrorString(e_));                \
    } while (0)

#define TRY(expr)                                                                       \
    do {                                                                                \
        int rc_ = (expr);                                                               \
        if (rc_ < 0) return rc_;                                                        \
    } while (0)

// ------------------------------------------------------------------ memory

void *dev_alloc(size_t bytes);
void dev_free(void *p, size_t bytes);
// While set on a thread, dev_alloc / dev_free use hipMalloc / hipFree even
// when an allocator is registered (server worker threads, which must not
// call back into the host application).
void set_thread_native_alloc(bool on);

// Workspace slots: each slot is a grow-only device buffer owned by the
// context, reused across calls.  A routine owns the slots listed for it.
enum WsSlot {
    WS_SCAN_L0 = 0,   // scan: block sums, 4 recursion levels
    WS_SCAN_L1,
    WS_SCAN_L2,
    WS_SCAN_L3,
    WS_SORT_TMP,      // radix sort ping-pong buffer
    WS_SORT_HIST,     // radix sort digit histograms
    WS_COUNTERS,      // small device counters
    WS_KEYS,          // build/relabel: 64-bit keys
    WS_FLAGS,         // build: dedup flags / positions
    WS_DEG,           // degrees, ordering
    WS_PERM,
    WS_BFS_A,         // BFS state
    WS_BFS_B,
    WS_BFS_C,
    WS_BFS_D,
    WS_BFS_E,
    WS_BC_SIGMA,      // BC state
    WS_BC_W,
    WS_BC_MASKS,
    WS_BC_UNVIS,
    WS_BC_ACT,        // BC active-vertex lists (two)
    WS_BC_CNT,        // BC per-level counters
    WS_GEN_A,         // generic operations
    WS_GEN_B,
    WS_GEN_C,
    WS_GEN_D,
    WS_GEN_E,
    WS_GEN_F,
    WS_GEN_G,
    WS_GEN_H,
    WS_TC,            // triangle counting
    WS_TC_WORK,
    WS_SSSP,          // SSSP device state
    WS_CHUNK_A,       // long-row chunk lists
    WS_CHUNK_B,
    WS_VXM_CAND,      // any.secondi push: per-output smallest index (kept all-ones)
    WS_VXM_UMAP,      // any.secondi: presence maps of sparse operands
    WS_VXM_MMAP,
    WS_VXM_LONG,      // any.secondi push: queued long rows
    WS_NSLOTS
};

struct KernelTimer {
    std::string name;
    hipEvent_t start, stop;
};

struct lagr_ctx_s {
    int timing = 0;
    std::vector<KernelTimer> timers;
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws[WS_NSLOTS] = {};
    size_t ws_bytes[WS_NSLOTS] = {};
    void *pinned = nullptr;          // pinned host staging for scalars: LAGR_PINNED_BYTES
    void *pinned_dev = nullptr;      // the same buffer's device address
    uint32_t host_seq = 0;           // last sequence number of a host wait
    int num_cus = 256;
    std::vector<void *> lvpool;      // per-level lane masks + vertex lists (BC)
    size_t lv_bytes = 0;
    // BFS: graphs of the search's start and first levels, and of further
    // levels, valid for bfs_key vertices and the state struct at
    // bfs_state, and the stream they are captured on
    hipGraphExec_t bfs_exec = nullptr;
    hipGraphExec_t bfs_exec_more = nullptr;
    hipGraph_t bfs_graph = nullptr;            // the first graph (its start node is updated per search)
    hipGraphNode_t bfs_start_node = nullptr;
    int64_t bfs_key = -1;
    void *bfs_state = nullptr;
    void *bfs_ctr = nullptr;
    // multi-source BFS: captured start and first levels, keyed by every
    // argument of their nodes
    hipGraphExec_t ms_exec = nullptr;
    std::vector<uintptr_t> ms_key;
    // SSSP: captured two-step graph, keyed the same way
    hipGraphExec_t sssp_exec = nullptr;
    int64_t sssp_key = -1;
    void *sssp_state = nullptr;
    hipStream_t capture_stream = nullptr;
    int64_t last_bc_levels = 0;       // levels of the deepest batch of the last bc_compute
    // any.secondi vxm: the WS_VXM_CAND buffer whose header (zero) and
    // first vxm_cand_n candidates (all ones) are in their between-call
    // state, and a spare pair of bitmap-vector arrays that the next result
    // on this stream takes (double buffering)
    void *vxm_cand = nullptr;
    int64_t vxm_cand_n = 0;
    uint8_t *vspare_present = nullptr;
    void *vspare_values = nullptr;
    size_t vspare_pb = 0, vspare_vb = 0;
    // device buffers that queued work may still read, freed at this
    // context's next wait for its stream (defer_free)
    std::vector<std::pair<void *, size_t>> deferred;
    size_t deferred_bytes = 0;
};

// Free p once the work queued so far on ctx's stream is done: at the
// context's next wait (lagr_wait, a read-back, a host wait), or at once
// after a stream sync when more than 2 GiB are pending.
void defer_free(lagr_ctx ctx, void *p, size_t bytes);
// Free everything deferred (the caller has waited for the stream).
void flush_deferred(lagr_ctx ctx);
// Device bytes a context holds between calls (workspace, level pool,
// spare vector arrays, deferred frees).
size_t ctx_retained_bytes(const lagr_ctx ctx);
// Wait for the stream and free all of it (and the captured graphs that
// point into it); later calls allocate again.
void ctx_trim(lagr_ctx ctx);

// Returns a device buffer of at least `bytes` for the slot (contents are
// undefined).  nullptr on allocation failure.
void *ws_get(lagr_ctx ctx, WsSlot slot, size_t bytes);

struct lagr_matrix_s {
    lagr_type type = LAGR_BOOL;
    int64_t nrows = 0, ncols = 0, nvals = 0;
    int64_t *rowptr = nullptr;
    int32_t *colidx = nullptr;
    void *values = nullptr;
    size_t rowptr_bytes = 0, colidx_bytes = 0, values_bytes = 0;  // 0 = borrowed
    // the transpose, built on the first call that asks for it with a
    // transpose descriptor and dropped with the arrays
    lagr_matrix_s *tcache = nullptr;
};

struct lagr_vector_s {
    lagr_type type = LAGR_BOOL;
    int64_t n = 0;
    lagr_vformat fmt = LAGR_VEC_SPARSE;
    int64_t nvals = 0;              // exact for SPARSE and FULL; -1 = unknown (BITMAP)
    int32_t *idx = nullptr;         // SPARSE
    uint8_t *present = nullptr;     // BITMAP
    void *values = nullptr;
    size_t idx_bytes = 0, present_bytes = 0, values_bytes = 0;      // 0 = borrowed
    // BITMAP only: a device word holding the entry count (in the tail of
    // the present array), kept by the operations that write it; nullptr:
    // count the presence bytes
    unsigned long long *count_dev = nullptr;
};

struct TcPlan;

// Owned chunk list of a matrix's long rows (n = -1: not built).
struct ChunkCache {
    int64_t n = -1;
    int32_t *row = nullptr;
    int64_t *beg = nullptr;
    int64_t *end = nullptr;
};

struct lagr_graph_s {
    lagr_matrix A = nullptr;
    lagr_kind kind = LAGR_ADJACENCY_UNDIRECTED;
    int64_t *row_degree = nullptr;  // cached property, int64[n]
    int64_t max_degree = -1;
    int64_t deg_over_sort = -1;     // vertices with more neighbours than the LDS row sort takes (with row_degree)
    int64_t ndiag = -1;             // -1 unknown
    int symmetric = -1;             // -1 unknown, 0 no, 1 yes
    lagr_matrix L = nullptr;        // degree-ordered strictly lower part
    int64_t L_maxrow = -1;
    // the plan's status (its counts, L's longest row) is still on the device,
    // in the context's counters, to be read with the first count
    bool tc_status_pending = false;
    // chunks of A's rows longer than GRAPH_LONG_ROW (owned arrays)
    ChunkCache chunks;
    // min-side triangle-count plan over L (built with L, owned)
    TcPlan *tcplan = nullptr;
    // transpose of A for a directed graph (the AT property, owned; an
    // undirected graph uses A itself) and the chunks of its long rows
    lagr_matrix AT = nullptr;
    ChunkCache chunks_t;
    // tuning settings (kept by lagr_graph_delete_properties): the count
    // plan's hub columns (-1: the default share of the vertices) and the
    // BFS direction thresholds
    int64_t tc_hubs = -1;
    int32_t bfs_alpha = 14, bfs_beta = 24;
};

// The pull side of G: AT for a directed graph (nullptr if not computed),
// A for an undirected one.
static inline lagr_matrix graph_in_edges(const lagr_graph G)
{
    return G->kind == LAGR_ADJACENCY_DIRECTED ? G->AT : G->A;
}

// Build / release G->tcplan from G->L, the row of each entry of L and the
// region starts of the plan's 2n virtual rows (regions: 2n+1 device int64,
// the exclusive scan of [row lengths of L | column lengths of L | 0]).
int tc_plan_build(lagr_ctx ctx, lagr_graph G, const int32_t *rowid, const int64_t *regions, char *msg);
// One host round trip after the build: status[0] (the longest row of L)
// and status[1] (rows left unsorted, *unsorted) come from the caller's
// kernels; sets G->L_maxrow and the plan's entry and item counts, and
// checks that L has nnz entries.
int tc_plan_settle(lagr_ctx ctx, lagr_graph G, unsigned long long *status, int64_t nnz, bool *unsorted,
                   char *msg);
// The same checks on a status already read back (st[0..5]).
int tc_plan_settle_host(lagr_graph G, const unsigned long long *st, int64_t nnz, bool *unsorted, char *msg);
// Launch the kernel that copies the plan's counts into status[3..5].
int tc_plan_status(lagr_ctx ctx, lagr_graph G, unsigned long long *status, char *msg);
// The triangle-count operand, for lagr_tc: with defer, and when the degrees
// prove every row of L short enough for the row sort, the plan's status is
// left on the device (G->tc_status_pending) for the count to read with its
// result.
int tc_lower_build(lagr_graph G, lagr_ctx ctx, bool defer, char *msg);
// Rows of L up to this many ids are sorted in LDS.
constexpr int64_t TC_SORT_LONG = 2048;
// Whether rows of max_row ids fit the count plan's length field.
bool tc_plan_fits(int64_t max_row);
void tc_plan_free(lagr_graph G);

// Rows of A longer than this are cut into chunks of this many entries for
// the BFS and BC kernels.
constexpr int64_t GRAPH_LONG_ROW = 512;


static inline size_t type_size(lagr_type t) { return t == LAGR_BOOL ? 0 : 8; }
// Bytes of one value in arrays that cross the boundary.
static inline size_t api_value_size(lagr_type t) { return t == LAGR_BOOL ? 0 : t == LAGR_INT32 ? 4 : 8; }
// int32 <-> the 8-byte slots the library keeps values in (n values).
int widen_i32(lagr_ctx ctx, const int32_t *src, int64_t *dst, int64_t n, char *msg);
int narrow_i64(lagr_ctx ctx, const int64_t *src, int32_t *dst, int64_t n, char *msg);

// Release a matrix's / vector's owned arrays and reset them to empty.
void matrix_release_arrays(lagr_matrix A);
void vector_release_arrays(lagr_vector v);
// The same, with the frees deferred until ctx's queued work is done.
void matrix_release_arrays_later(lagr_ctx ctx, lagr_matrix A);
void vector_release_arrays_later(lagr_ctx ctx, lagr_vector v);
// Entries of a presence-byte map (synchronises).
int bitmap_count(lagr_ctx ctx, const uint8_t *present, int64_t n, int64_t *count, char *msg);
// vxm with any.secondi under a complemented structural mask with replace
// (push, or pull with TRAN1), optionally assigning the parents into the
// mask: 1 when served, 0 when the call has another shape, < 0 on error.
int vxm_any_secondi_fast(lagr_vector w, lagr_vector m, lagr_binop accum, lagr_semiring semiring,
                         const lagr_vector u, const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg);
// Allocate owned arrays for a CSR of the given size (rowptr always).
int matrix_alloc(lagr_matrix A, int64_t nvals, char *msg);

// Kernel timing: TIMED_LAUNCH(ctx, "name", launch-expression)
void timer_begin(lagr_ctx ctx, const char *name, hipEvent_t *stop);
void timer_end(lagr_ctx ctx, hipEvent_t stop);
#define TIMED(ctx, name, ...)                                   \
    do {                                                        \
        hipEvent_t stop_ev_ = nullptr;                          \
        if ((ctx)->timing) timer_begin((ctx), (name), &stop_ev_);\
        __VA_ARGS__;                                            \
        if (stop_ev_) timer_end((ctx), stop_ev_);               \
    } while (0)

// ------------------------------------------------------------- primitives

// Exclusive prefix sum of int64 in[0..n) into out (may alias in).  If
// total != nullptr the grand total is copied to the host (synchronises).
int scan_exclusive_i64(lagr_ctx ctx, const int64_t *in, int64_t *out, int64_t n,
                       int64_t *total, char *msg);
// Stable LSD radix sort of n 64-bit keys on bits [0, nbits), in place.
int radix_sort_u64(lagr_ctx ctx, uint64_t *keys, int64_t n, int nbits, char *msg);
// Fill helpers (graph-capture safe, no hipMemset).
int fill_i64(lagr_ctx ctx, int64_t *p, int64_t n, int64_t value, char *msg);
int fill_u32(lagr_ctx ctx, uint32_t *p, int64_t n, uint32_t value, char *msg);
int fill_u8(lagr_ctx ctx, uint8_t *p, int64_t n, uint8_t value, char *msg);
// The pinned buffer: LAGR_PINNED_STAGE bytes of staging for read_back and
// stage_to_host, then LAGR_PINNED_FLAGS bytes of flags that kernels store
// to directly: the BFS level loop's done flag at LAGR_PINNED_STAGE and the
// sequence word of host waits at LAGR_PINNED_SEQ.
// The BFS level loop also stores the index of the level that has started
// at LAGR_PINNED_LEVEL.
constexpr size_t LAGR_PINNED_STAGE = 4096;
constexpr size_t LAGR_PINNED_LEVEL = LAGR_PINNED_STAGE + 8;
constexpr size_t LAGR_PINNED_SEQ = LAGR_PINNED_STAGE + 64;
constexpr size_t LAGR_PINNED_FLAGS = 256;
constexpr size_t LAGR_PINNED_BYTES = LAGR_PINNED_STAGE + LAGR_PINNED_FLAGS;
// Enqueue a copy of `bytes` device bytes to the pinned buffer at `offset`
// (a one-workgroup kernel storing to the buffer's device address when both
// are 4-byte multiples, which costs less than the runtime's copy; else
// hipMemcpyAsync).  With wait, return once the copy and all earlier work
// on the stream are done (the kernel stores a sequence number after the
// words and the host polls it); without, the host reads the buffer only
// after a later wait.
int stage_to_host(lagr_ctx ctx, size_t offset, const void *dev, size_t bytes, bool wait, char *msg);
// Return once all work enqueued on the context's stream is done (the same
// polled sequence number, with no words).
int host_wait(lagr_ctx ctx, char *msg);
// Copy a few bytes device -> host through the context's pinned buffer and
// wait for the stream.
int read_back(lagr_ctx ctx, void *host, const void *dev, size_t bytes, char *msg);
// Build CSR row offsets (n+1) from row ids of `nnz` sorted keys whose row
// is key >> shift.
int rowptr_from_sorted_keys(lagr_ctx ctx, const uint64_t *keys, int64_t nnz, int shift,
                            int64_t nrows, int64_t *rowptr, char *msg);
// Chunks of the rows longer than `min_len` entries, each at most `chunk`
// entries, so that a hub row is spread over many wavefronts.  The arrays
// live in the two workspace slots given; n is on the host (synchronises).
struct RowChunks {
    int64_t n;
    const int32_t *row;
    const int64_t *beg;
    const int64_t *end;
};
int row_chunks(lagr_ctx ctx, const int64_t *rowptr, int64_t nrows, int64_t min_len, int64_t chunk,
               WsSlot count_slot, WsSlot list_slot, RowChunks *out, char *msg);
// The cached chunk list of G->A (built on first use).
int graph_chunks(lagr_graph G, lagr_ctx ctx, RowChunks *out, char *msg);
// The cached chunk list of the pull side, graph_in_edges(G) (which must
// exist).
int graph_chunks_in(lagr_graph G, lagr_ctx ctx, RowChunks *out, char *msg);
// A new matrix holding the transpose of A (values carried), owned by the
// caller.
int matrix_transpose(lagr_ctx ctx, const lagr_matrix A, lagr_matrix *out, char *msg);
// Compute G->AT for a directed graph if it is missing (no-op otherwise).
int graph_ensure_at(lagr_graph G, lagr_ctx ctx, char *msg);
// Betweenness of 64-lane batches (lane_src: HOST, 64 per batch, -1 idle)
// into cent: gshift 6 sums all lanes (n values), gshift 3 sums groups of 8
// lanes (n x 8 values).  backward: BC_BACKWARD_PULL (fixed order: the
// same bits every run), BC_BACKWARD_AUTO (push or pull per level) or
// BC_BACKWARD_PUSH (push on every level).
enum { BC_BACKWARD_PULL = 0, BC_BACKWARD_AUTO = 1, BC_BACKWARD_PUSH = 2 };
int bc_compute(lagr_ctx ctx, const lagr_graph G, const int64_t *lane_src, int nbatches, int gshift,
               double *cent, char *msg, int backward = BC_BACKWARD_PULL);
// Multi-source BFS of up to 64 lanes (lane_src: HOST, 64, -1 idle): per
// lane reached count, level sum and depth into stats[3][64] (host); with
// lev (n x 64 uint16), the level of every reached (vertex, lane), 0xFFFF
// elsewhere.
int msbfs_compute(lagr_ctx ctx, const lagr_graph G, const int64_t *lane_src, uint16_t *lev, int64_t *stats,
                  char *msg);
// Row degrees (rowptr differences) into deg[n], their maximum and the number
// above `big` (host).
int row_degrees(lagr_ctx ctx, const int64_t *rowptr, int64_t n, int64_t *deg,
                int64_t *maxdeg, char *msg, int64_t big = INT64_MAX, int64_t *nbig = nullptr);

static inline int bits_for(uint64_t x)
{
    int b = 0;
    while (b < 64 && (x >> b) != 0) b++;
    return b;
}

static inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 20)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Device helpers ----------------------------------------------------------

__device__ __forceinline__ unsigned lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Chunks of the rows whose vertex is set in bitmap bm, for a kernel whose
// wavefronts share the chunk list: each lane tests one chunk (64 tests in
// flight per wave instead of one dependent test per chunk), and chunk
// indices interleave across wavefronts (lane l of wave w tests chunk
// w + (l + 64 k) nw), so the consecutive chunks of one hub row spread over
// many wavefronts.  body(u, beg, end) runs with the whole wave for each
// hit.
template <typename Body>
__device__ __forceinline__ void for_marked_chunks(const RowChunks &ch, const uint32_t *__restrict__ bm,
                                                  Body body)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const unsigned lane = lane_id();
    for (int64_t k0 = 0; wave + k0 * nw < ch.n; k0 += 64) {
        const int64_t c = wave + (k0 + lane) * nw;
        bool hit = false;
        if (c < ch.n) {
            const int32_t u = ch.row[c];
            hit = (bm[u >> 5] >> (u & 31)) & 1u;
        }
        for (uint64_t m = __ballot(hit); m; m &= m - 1) {
            const int64_t cc = wave + (k0 + (int64_t)__ffsll((unsigned long long)m) - 1) * nw;
            body(ch.row[cc], ch.beg[cc], ch.end[cc]);
        }
    }
}

// For entries in row order, one per lane: the lanes of the wave whose key
// (row) equals this lane's form one contiguous run.  The run's first lane
// (head) can make one atomic on the row's counter for the whole run (atomics
// from many lanes on one address are serialised).  run: the lanes of the
// run; before: those of them below this lane.  Every lane of the wave must
// call it.
// Inclusive sum over the 64 lanes by DPP moves (no LDS round trip):
// Hillis-Steele steps of 1, 2, 4 and 8 lanes within each 16-lane row
// (row_shr; a lane with no source lane adds 0), then the end of row 0 into
// rows 1 and 3 and the end of row 1 (now rows 0-1) into rows 2 and 3
// (row_bcast:15 / :31 with row masks 0xa / 0xc).  Every lane must be active.
__device__ __forceinline__ int wave_incl_sum(int x)
{
    int t = x;
    t += __builtin_amdgcn_update_dpp(0, t, 0x111, 0xf, 0xf, false);   // row_shr:1
    t += __builtin_amdgcn_update_dpp(0, t, 0x112, 0xf, 0xf, false);   // row_shr:2
    t += __builtin_amdgcn_update_dpp(0, t, 0x114, 0xf, 0xf, false);   // row_shr:4
    t += __builtin_amdgcn_update_dpp(0, t, 0x118, 0xf, 0xf, false);   // row_shr:8
    t += __builtin_amdgcn_update_dpp(0, t, 0x142, 0xa, 0xf, false);   // row_bcast:15
    t += __builtin_amdgcn_update_dpp(0, t, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return t;
}

// Exclusive prefix of x over a block of 256 threads (in thread order) and
// the block total: DPP sums within the waves, then the four wave totals
// through LDS (wtot, 4 entries).  Every thread of the block must call it;
// wtot may be reused after the next __syncthreads.
__device__ __forceinline__ unsigned block_excl_scan256(unsigned x, unsigned *wtot, unsigned &total)
{
    const unsigned lane = lane_id(), w = threadIdx.x >> 6;
    const unsigned incl = (unsigned)wave_incl_sum((int)x);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    unsigned before = 0, all = 0;
#pragma unroll
    for (unsigned k = 0; k < 4; k++) {
        const unsigned t = wtot[k];
        before += k < w ? t : 0u;
        all += t;
    }
    total = all;
    return before + incl - x;
}

// A 64-bit value moved by one DPP control (both halves; 0 where the
// source lane is missing or the row is masked off).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, ROW_MASK, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// The sum of x over the 64 lanes (every lane active), by the steps of
// wave_incl_sum on 64-bit values; the total is read from lane 63.
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x)
{
    x += dpp_u64<0x111, 0xf>(x);   // row_shr:1
    x += dpp_u64<0x112, 0xf>(x);   // row_shr:2
    x += dpp_u64<0x114, 0xf>(x);   // row_shr:4
    x += dpp_u64<0x118, 0xf>(x);   // row_shr:8
    x += dpp_u64<0x142, 0xa>(x);   // row_bcast:15
    x += dpp_u64<0x143, 0xc>(x);   // row_bcast:31
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

struct WaveRun {
    unsigned head;
    uint64_t run, before;
};

__device__ __forceinline__ WaveRun wave_run(int32_t key)
{
    const unsigned lane = lane_id();
    // the previous lane's key by a DPP wave shift (wave_shr:1; lane 0 has
    // none and is a head anyway)
    const int32_t prev = __builtin_amdgcn_update_dpp(0, key, 0x138, 0xf, 0xf, false);
    const uint64_t H = __ballot(lane == 0 || prev != key);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    WaveRun w;
    w.head = 63 - __clzll((unsigned long long)(H & upto));
    const uint64_t after = H & ~upto;
    const uint64_t hi = after ? ((1ull << (__ffsll((unsigned long long)after) - 1)) - 1) : ~0ull;
    w.run = hi & ~((1ull << w.head) - 1);
    w.before = w.run & ((1ull << lane) - 1);
    return w;
}
