// The BFS-shaped vxm calls of the GraphBLAS form, on their own kernels:
//
//   w<!s(m), replace> = u any.secondi A'          (Algorithm 1's step; push)
//   w<!s(m), replace> = u any.secondi A', A' = S^T (the pull form, TRAN1)
//
// optionally fused with the parent assignment m<s(w)> = w (the
// LAGR_DESC_ASSIGN_PARENT extension: the mask is the parent vector p of
// Algorithms 1-2, Section IV-A; the fusion is the one Section VI-B says a
// non-blocking library may do).  secondi(u_k, a_kj) = k, and the any
// monoid returns the smallest admissible k, as on every other path of this
// library, so push and pull give the same result.
//
// The result is a BITMAP vector (presence byte per index, int64 values)
// whose entry count is kept in a device word: no call here waits for the
// stream or allocates in steady state.  The result's arrays come from a
// spare pair kept by the context, and w's previous arrays become the spare
// (double buffering: w may be u or m, as in q = q any.secondi A); arrays
// that leave are freed once the queued kernels are done (defer_free).
//
// Push: each wavefront takes 64 frontier vertices k (list entries of a
// SPARSE u, or 64 consecutive indices of a bitmap or full u) and spreads
// the entries of their rows of A over its lanes; rows longer than LONG_ROW
// are queued and walked by the whole grid in a second kernel.  Every entry
// (k, j) with j outside s(m) takes cand[j] = min(cand[j], k) with a
// no-return atomic.  A finishing pass over
// the n outputs turns cand into w (and p), counts the entries and puts
// cand back to all ones, so it never needs a separate clear.
// Pull: one lane per output j outside s(m) walks row j of the stored
// matrix S until the first k present in u (rows are sorted, so that is the
// smallest) and writes w(j) (and p(j)) itself.
#include "internal.h"

#include <climits>

namespace {

constexpr uint32_t NO_K = 0xffffffffu;

struct VxmArgs {
    const int64_t *rp;        // rows of the stored matrix
    const int32_t *ci;
    int64_t nk;               // u's length
    int64_t nw;               // w's length
    // u: list (SPARSE), presence bytes (BITMAP) or all present (FULL)
    int ulist;
    const int32_t *uidx;
    int64_t unv;
    const uint8_t *upres;
    int ufull;
    // mask: presence bytes, or full
    const uint8_t *mpres;
    int mfull;
    // outputs
    uint8_t *wpres;
    int64_t *wval;
    unsigned long long *wcount;
    int assign;
    uint8_t *ppres;           // the mask's own arrays (parent assignment)
    int64_t *pval;
    unsigned long long *pcount;
    uint32_t *cand;
    unsigned *nlong;          // queued long-row chunks (push), zeroed by k_vxm_finish
    uint64_t *longq;
    unsigned longcap;
};

// Rows longer than LONG_ROW go to a queue of LONG_ROW-entry chunks that
// the whole grid walks next, one wavefront per chunk.  A chunk is queued as
// (row << 20) | chunk index (rows have fewer than 2^31 entries, so fewer
// than 2^20 chunks); the queue holds at most nnz(A) / 1024 chunks (a long
// row of len entries makes ceil(len / LONG_ROW) < 2 len / LONG_ROW).
constexpr int64_t LONG_ROW = 2048;

__device__ __forceinline__ void push_entry(const VxmArgs &a, int64_t p, uint32_t k)
{
    const int32_t j = a.ci[p];
    if (a.mpres[j]) return;                 // (a full mask returns before this)
    __hip_atomic_fetch_min(a.cand + j, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Each wavefront takes 64 frontier vertices (list entries, or 64
// consecutive indices of a bitmap / full u), one per lane, and spreads the
// entries of their rows over its lanes: an in-wave prefix sum of the row
// lengths lays the rows end to end in LDS (offsets, row starts, indices),
// and lane l takes entries t = l, l + 64, ... of the batch, walking the
// offsets forward to the row that holds t (its entries only increase: one
// step per row boundary crossed).  VXM_DEPTH entries per lane go through
// each stage together (their ids, then their mask bytes, then their
// atomics).  A long row is queued.
constexpr int VXM_DEPTH = 4;

__global__ __launch_bounds__(256) void k_vxm_push(const VxmArgs a)
{
    __shared__ int32_t s_off[4][65];
    __shared__ int64_t s_b[4][64], s_k[4][64];
    const int lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.wcount = 0;
    if (a.mfull) return;                    // every output is masked out
    const int64_t nitems = a.ulist ? a.unv : a.nk;
    for (int64_t base = wave * 64; base < nitems; base += nwaves * 64) {
        const int64_t q = base + lane;
        int64_t k = -1;
        if (q < nitems) {
            if (a.ulist) k = a.uidx[q];
            else if (a.ufull || a.upres[q]) k = q;
        }
        int64_t b = 0;
        int32_t len = 0;
        if (k >= 0) {
            b = a.rp[k];
            const int64_t l = a.rp[k + 1] - b;
            if (l > LONG_ROW) {
                const unsigned nc = (unsigned)((l + LONG_ROW - 1) / LONG_ROW);
                const unsigned slot = atomicAdd(a.nlong, nc);
                // (the bound holds for a vector's distinct indices; the
                // check keeps repeated indices of a wrapped list in bounds)
                for (unsigned c = 0; c < nc; c++)
                    if (slot + c < a.longcap) a.longq[slot + c] = ((uint64_t)k << 20) | c;
            } else {
                len = (int32_t)l;
            }
        }
        // inclusive prefix of len over the wave
        const int32_t inc = wave_incl_sum(len);
        const int32_t total = __builtin_amdgcn_readlane(inc, 63);
        if (total == 0) continue;
        s_off[wib][lane + 1] = inc;
        if (lane == 0) s_off[wib][0] = 0;
        s_b[wib][lane] = b - (inc - len);   // row start minus the row's offset in the batch
        s_k[wib][lane] = k;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the lane's row r (offsets s_off[r] <= t < rend = s_off[r + 1]),
        // its start minus offset rb and index rk, in registers
        int r = 0, rend = s_off[wib][1];
        int64_t rb = s_b[wib][0], rk = s_k[wib][0];
        for (int32_t t0 = 0; t0 < total; t0 += 64 * VXM_DEPTH) {
            int64_t pp[VXM_DEPTH];
            uint32_t kk[VXM_DEPTH];
#pragma unroll
            for (int dd = 0; dd < VXM_DEPTH; dd++) {
                const int32_t t = t0 + 64 * dd + lane;
                pp[dd] = -1;
                kk[dd] = 0;
                if (t < total) {
                    if (rend <= t) {
                        do {
                            ++r;
                            rend = s_off[wib][r + 1];
                        } while (rend <= t);
                        rb = s_b[wib][r];
                        rk = s_k[wib][r];
                    }
                    pp[dd] = rb + t;
                    kk[dd] = (uint32_t)rk;
                }
            }
            int32_t jj[VXM_DEPTH];
#pragma unroll
            for (int dd = 0; dd < VXM_DEPTH; dd++) jj[dd] = pp[dd] >= 0 ? a.ci[pp[dd]] : -1;
            uint8_t mp[VXM_DEPTH];
#pragma unroll
            for (int dd = 0; dd < VXM_DEPTH; dd++) mp[dd] = jj[dd] >= 0 ? a.mpres[jj[dd]] : (uint8_t)1;
#pragma unroll
            for (int dd = 0; dd < VXM_DEPTH; dd++)
                if (!mp[dd]) __hip_atomic_fetch_min(a.cand + jj[dd], kk[dd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// The queued chunks of long rows, one wavefront per chunk.
__global__ __launch_bounds__(256) void k_vxm_push_long(const VxmArgs a)
{
    const unsigned nl = *a.nlong < a.longcap ? *a.nlong : a.longcap;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < nl; r += nwaves) {
        const uint64_t q = a.longq[r];
        const int64_t k = (int64_t)(q >> 20);
        const int64_t b = a.rp[k] + (int64_t)(q & 0xfffff) * LONG_ROW;
        const int64_t re = a.rp[k + 1];
        const int64_t e = b + LONG_ROW < re ? b + LONG_ROW : re;
        for (int64_t p = b + lane; p < e; p += 64) push_entry(a, p, (uint32_t)k);
    }
}

// block sum of one 0/1 flag per thread, added to the counters by thread 0
__device__ __forceinline__ void add_count(unsigned c, unsigned long long *w, unsigned long long *p)
{
    __shared__ unsigned s[4];
    const unsigned long long bal = __ballot(c != 0);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = (unsigned)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = (unsigned long long)s[0] + s[1] + s[2] + s[3];
        if (t) {
            atomicAdd(w, t);
            if (p) atomicAdd(p, t);
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_vxm_finish(const VxmArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t end = (a.nw + 255) / 256 * 256;       // whole blocks: every thread reaches add_count
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.nlong = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < end; j += stride) {
        unsigned hit = 0;
        if (j < a.nw) {
            const uint32_t c = a.cand[j];
            hit = c != NO_K;
            a.wpres[j] = (uint8_t)hit;
            if (hit) {
                a.wval[j] = (int64_t)c;
                a.cand[j] = NO_K;
                if (a.assign) {
                    a.ppres[j] = 1;
                    a.pval[j] = (int64_t)c;
                }
            }
        }
        add_count(hit, a.wcount, a.assign ? a.pcount : nullptr);
    }
}

__global__ __launch_bounds__(256) void k_vxm_pull(const VxmArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t end = (a.nw + 255) / 256 * 256;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < end; j += stride) {
        unsigned hit = 0;
        if (j < a.nw) {
            int64_t k = -1;
            if (!a.mfull && !a.mpres[j]) {
                const int64_t b = a.rp[j], e = a.rp[j + 1];
                for (int64_t p = b; p < e; p++) {
                    const int32_t c = a.ci[p];
                    if (a.ufull || a.upres[c]) {
                        k = c;
                        break;
                    }
                }
            }
            hit = k >= 0;
            a.wpres[j] = (uint8_t)hit;
            if (hit) {
                a.wval[j] = k;
                if (a.assign) {
                    a.ppres[j] = 1;
                    a.pval[j] = k;
                }
            }
        }
        add_count(hit, a.wcount, a.assign ? a.pcount : nullptr);
    }
}

__global__ void k_set_word(unsigned long long *w, unsigned long long v) { *w = v; }

__global__ void k_scatter_list(const int32_t *__restrict__ idx, const int64_t *__restrict__ vals, int64_t nv,
                               uint8_t *__restrict__ pres, int64_t *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv; q += (int64_t)gridDim.x * blockDim.x) {
        pres[idx[q]] = 1;
        if (out) out[idx[q]] = vals[q];
    }
}

// Presence bytes of n entries plus the count word after them (8-aligned).
size_t present_bytes_for(int64_t n) { return ((size_t)(n > 0 ? n : 1) + 7) / 8 * 8 + 8; }

unsigned long long *count_word(uint8_t *present, int64_t n)
{
    return (unsigned long long *)(present + ((size_t)(n > 0 ? n : 1) + 7) / 8 * 8);
}

// A presence map of a SPARSE vector in a workspace slot.
int sparse_map(lagr_ctx ctx, const lagr_vector v, WsSlot slot, const uint8_t **map, char *msg)
{
    uint8_t *m = (uint8_t *)ws_get(ctx, slot, (size_t)(v->n > 0 ? v->n : 1));
    if (!m) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "presence map");
    TRY(fill_u8(ctx, m, v->n, 0, msg));
    if (v->nvals > 0) {
        hipLaunchKernelGGL(k_scatter_list, dim3(grid_for(v->nvals, 256, 16384)), dim3(256), 0, ctx->stream, v->idx,
                           (const int64_t *)nullptr, v->nvals, m, (int64_t *)nullptr);
        LAUNCH_CHECK();
    }
    *map = m;
    return LAGR_SUCCESS;
}

// Turn the parent vector p (SPARSE or FULL, INT64) into an owned BITMAP
// with a count word, in place.
int parent_to_bitmap(lagr_ctx ctx, lagr_vector p, char *msg)
{
    const int64_t n = p->n;
    const size_t pb = present_bytes_for(n), vb = 8 * (size_t)(n > 0 ? n : 1);
    uint8_t *pres = (uint8_t *)dev_alloc(pb);
    int64_t *vals = (int64_t *)dev_alloc(vb);
    if (!pres || !vals) {
        dev_free(pres, pb);
        dev_free(vals, vb);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "parent arrays");
    }
    unsigned long long *cw = count_word(pres, n);
    int64_t count = 0;
    if (p->fmt == LAGR_VEC_FULL) {
        TRY(fill_u8(ctx, pres, n, 1, msg));
        if (n > 0) HIP_TRY(hipMemcpyAsync(vals, p->values, 8 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
        count = n;
    } else if (p->fmt == LAGR_VEC_SPARSE) {
        TRY(fill_u8(ctx, pres, n, 0, msg));
        if (p->nvals > 0) {
            hipLaunchKernelGGL(k_scatter_list, dim3(grid_for(p->nvals, 256, 16384)), dim3(256), 0, ctx->stream,
                               p->idx, (const int64_t *)p->values, p->nvals, pres, vals);
            LAUNCH_CHECK();
        }
        count = p->nvals;
    } else {
        // an uncounted or borrowed bitmap: copy, then count once
        HIP_TRY(hipMemcpyAsync(pres, p->present, (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
        if (n > 0) HIP_TRY(hipMemcpyAsync(vals, p->values, 8 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
        TRY(bitmap_count(ctx, p->present, n, &count, msg));
    }
    hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, ctx->stream, cw, (unsigned long long)count);
    LAUNCH_CHECK();
    vector_release_arrays_later(ctx, p);
    p->fmt = LAGR_VEC_BITMAP;
    p->present = pres;
    p->present_bytes = pb;
    p->values = vals;
    p->values_bytes = vb;
    p->nvals = -1;
    p->count_dev = cw;
    return LAGR_SUCCESS;
}

}  // namespace

// Returns 1 and computes the product when the call has the shape this file
// serves, 0 (doing nothing) when it has not, < 0 on error.  The caller has
// validated arguments, dimensions and domains.
int vxm_any_secondi_fast(lagr_vector w, lagr_vector m, lagr_binop accum, lagr_semiring semiring,
                         const lagr_vector u, const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg)
{
    const uint32_t rsc = LAGR_DESC_REPLACE | LAGR_DESC_STRUCT | LAGR_DESC_COMP;
    const bool assign = desc & LAGR_DESC_ASSIGN_PARENT;
    if (semiring != LAGR_ANY_SECONDI || accum != LAGR_NOOP || !m || (desc & rsc) != rsc) return 0;
    if (w->type != LAGR_INT64 || w->n > INT32_MAX || ctx->device < 0) return 0;
    if (assign && (m == w || m == u || m->type != LAGR_INT64)) return 0;
    const bool pull = desc & LAGR_DESC_TRAN1;
    const int64_t nw = w->n;

    VxmArgs a{};
    a.rp = A->rowptr;
    a.ci = A->colidx;
    a.nk = u->n;
    a.nw = nw;
    a.assign = assign ? 1 : 0;

    // the mask (the parent vector when assigning)
    if (assign && (m->fmt != LAGR_VEC_BITMAP || !m->count_dev || !m->present_bytes))
        TRY(parent_to_bitmap(ctx, m, msg));
    if (m->fmt == LAGR_VEC_FULL) {
        a.mfull = 1;
    } else if (m->fmt == LAGR_VEC_BITMAP) {
        a.mpres = m->present;
    } else {
        TRY(sparse_map(ctx, m, WS_VXM_MMAP, &a.mpres, msg));
    }
    if (assign) {
        a.ppres = m->present;
        a.pval = (int64_t *)m->values;
        a.pcount = m->count_dev;
    }

    // u
    if (u->fmt == LAGR_VEC_FULL) {
        a.ufull = 1;
    } else if (u->fmt == LAGR_VEC_BITMAP) {
        a.upres = u->present;
    } else if (pull) {
        TRY(sparse_map(ctx, u, WS_VXM_UMAP, &a.upres, msg));
    } else {
        a.ulist = 1;
        a.uidx = u->idx;
        a.unv = u->nvals;
    }

    // w's new arrays: the context's spare pair when it fits
    const size_t pb = present_bytes_for(nw), vb = 8 * (size_t)(nw > 0 ? nw : 1);
    uint8_t *wp = nullptr;
    int64_t *wv = nullptr;
    if (ctx->vspare_present && ctx->vspare_pb == pb && ctx->vspare_vb == vb) {
        wp = ctx->vspare_present;
        wv = (int64_t *)ctx->vspare_values;
        ctx->vspare_present = nullptr;
        ctx->vspare_values = nullptr;
        ctx->vspare_pb = ctx->vspare_vb = 0;
    } else {
        wp = (uint8_t *)dev_alloc(pb);
        wv = (int64_t *)dev_alloc(vb);
        if (!wp || !wv) {
            dev_free(wp, pb);
            dev_free(wv, vb);
            return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vxm result arrays");
        }
    }
    a.wpres = wp;
    a.wval = wv;
    a.wcount = count_word(wp, nw);

    int rc = LAGR_SUCCESS;
    if (pull) {
        hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, ctx->stream, a.wcount, 0ull);
        hipLaunchKernelGGL(k_vxm_pull, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, ctx->stream, a);
    } else {
        // The buffer holds a 64-word header, whose first word is the
        // long-row chunk count, then cand.  Between calls the count is
        // zero and cand all ones (the finishing pass restores both); a new
        // buffer gets both once, and a longer output its new cand entries.
        const int64_t ncand = (nw + 63) / 64 * 64;
        uint32_t *buf = (uint32_t *)ws_get(ctx, WS_VXM_CAND, 4 * (size_t)(64 + ncand));
        uint32_t *cand = buf ? buf + 64 : nullptr;
        uint64_t *longq = (uint64_t *)ws_get(ctx, WS_VXM_LONG, 8 * (size_t)(A->nvals / 1024 + 64));
        if (!cand || !longq) rc = lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vxm candidates");
        if (rc == LAGR_SUCCESS && (buf != ctx->vxm_cand || ctx->vxm_cand_n < nw)) {
            if (buf != ctx->vxm_cand) rc = fill_u32(ctx, buf, 64, 0u, msg);
            ctx->vxm_cand = nullptr;
            ctx->vxm_cand_n = 0;
            if (rc == LAGR_SUCCESS) rc = fill_u32(ctx, cand, ncand, NO_K, msg);
            if (rc == LAGR_SUCCESS) {
                ctx->vxm_cand = buf;
                ctx->vxm_cand_n = ncand;
            }
        }
        if (rc == LAGR_SUCCESS) {
            a.cand = cand;
            a.nlong = buf;
            a.longq = longq;
            a.longcap = (unsigned)(A->nvals / 1024 + 64);
            // a full mask admits no output: the push kernel only clears
            // the count (it has no mpres to read)
            const int64_t items = a.mfull ? 0 : a.ulist ? a.unv : u->n;
            hipLaunchKernelGGL(k_vxm_push, dim3(grid_for(items, 256, 8192)), dim3(256), 0, ctx->stream, a);
            if (!a.mfull && A->nvals > LONG_ROW)
                hipLaunchKernelGGL(k_vxm_push_long, dim3(2048), dim3(256), 0, ctx->stream, a);
            hipLaunchKernelGGL(k_vxm_finish, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, ctx->stream, a);
        }
    }
    if (rc == LAGR_SUCCESS && hipGetLastError() != hipSuccess)
        rc = lagr_fail(msg, LAGR_DEVICE_ERROR, "vxm launch");
    if (rc < 0) {
        dev_free(wp, pb);
        dev_free(wv, vb);
        return rc;
    }

    // w's old arrays become the spare (kernels queued above still read
    // them; the next user of the spare is later on the same stream)
    if (w->fmt == LAGR_VEC_BITMAP && w->present_bytes == pb && w->values_bytes == vb) {
        defer_free(ctx, ctx->vspare_present, ctx->vspare_pb);
        defer_free(ctx, ctx->vspare_values, ctx->vspare_vb);
        ctx->vspare_present = w->present;
        ctx->vspare_values = w->values;
        ctx->vspare_pb = pb;
        ctx->vspare_vb = vb;
        w->present = nullptr;
        w->values = nullptr;
        w->present_bytes = w->values_bytes = 0;
    }
    vector_release_arrays_later(ctx, w);
    w->fmt = LAGR_VEC_BITMAP;
    w->present = wp;
    w->present_bytes = pb;
    w->values = wv;
    w->values_bytes = vb;
    w->nvals = -1;
    w->count_dev = a.wcount;
    return 1;
}
