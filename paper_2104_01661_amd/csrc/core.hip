// Context, allocator, messages and the matrix / vector / graph objects.
#include <new>

#include "internal.h"

// ------------------------------------------------------------- messages

int lagr_fail(char *msg, int code, const char *fmt, ...)
{
    if (msg) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, LAGR_MSG_LEN, fmt, ap);
        va_end(ap);
    }
    return code;
}

static void timers_clear(lagr_ctx ctx);

// ------------------------------------------------------------- allocator

static lagr_alloc_fn g_alloc = nullptr;
static lagr_free_fn g_free = nullptr;
static void *g_user = nullptr;

static thread_local bool t_native_alloc = false;

void set_thread_native_alloc(bool on) { t_native_alloc = on; }

void *dev_alloc(size_t bytes)
{
    if (bytes == 0) return nullptr;
    if (g_alloc && !t_native_alloc) return g_alloc(bytes, g_user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_free(void *p, size_t bytes)
{
    if (!p) return;
    if (g_free && !t_native_alloc) {
        g_free(p, bytes, g_user);
        return;
    }
    (void)hipFree(p);
}

extern "C" int lagr_set_allocator(lagr_alloc_fn alloc, lagr_free_fn release, void *user, char *msg)
{
    if ((alloc == nullptr) != (release == nullptr))
        return lagr_fail(msg, LAGR_NULL_POINTER, "allocator and release must both be set or both NULL");
    g_alloc = alloc;
    g_free = release;
    g_user = user;
    return lagr_ok(msg);
}

// ------------------------------------------------------------- context

extern "C" int lagr_ctx_new(lagr_ctx *ctx, int device, void *stream, char *msg)
{
    if (!ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "ctx is NULL");
    *ctx = nullptr;
    if (device == -1) {
        // validation-only context: no device work can be queued on it, but
        // every argument check can run (it is what host-side tests use)
        lagr_ctx c = new (std::nothrow) lagr_ctx_s();
        if (!c) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "context");
        c->device = -1;
        *ctx = c;
        return lagr_ok(msg);
    }
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    lagr_ctx c = new (std::nothrow) lagr_ctx_s();
    if (!c) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "context");
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipHostMalloc(&c->pinned, LAGR_PINNED_BYTES, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "pinned staging buffer");
    }
    if (hipHostGetDevicePointer(&c->pinned_dev, c->pinned, 0) != hipSuccess || !c->pinned_dev) {
        (void)hipHostFree(c->pinned);
        delete c;
        return lagr_fail(msg, LAGR_DEVICE_ERROR, "pinned staging buffer: no device address");
    }
    memset(c->pinned, 0, LAGR_PINNED_BYTES);   // the flags start clear
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cus = prop.multiProcessorCount;
    *ctx = c;
    return lagr_ok(msg);
}

extern "C" int lagr_ctx_set_stream(lagr_ctx ctx, void *stream, char *msg)
{
    if (!ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "ctx is NULL");
    // work a call left queued (a search's last levels) finishes on the old
    // stream before the context's next work starts on the new one
    if (ctx->device >= 0 && ctx->stream != (hipStream_t)stream) {
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        flush_deferred(ctx);
    }
    ctx->stream = (hipStream_t)stream;
    return lagr_ok(msg);
}

extern "C" int lagr_ctx_free(lagr_ctx *ctx)
{
    if (!ctx || !*ctx) return LAGR_SUCCESS;
    lagr_ctx c = *ctx;
    if (c->device >= 0) (void)hipStreamSynchronize(c->stream);
    if (c->bfs_exec) (void)hipGraphExecDestroy(c->bfs_exec);
    if (c->bfs_exec_more) (void)hipGraphExecDestroy(c->bfs_exec_more);
    if (c->bfs_graph) (void)hipGraphDestroy(c->bfs_graph);
    if (c->sssp_exec) (void)hipGraphExecDestroy(c->sssp_exec);
    if (c->ms_exec) (void)hipGraphExecDestroy(c->ms_exec);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    timers_clear(c);
    for (int s = 0; s < WS_NSLOTS; s++) dev_free(c->ws[s], c->ws_bytes[s]);
    flush_deferred(c);
    for (void *p : c->lvpool) dev_free(p, c->lv_bytes);
    dev_free(c->vspare_present, c->vspare_pb);
    dev_free(c->vspare_values, c->vspare_vb);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    *ctx = nullptr;
    return LAGR_SUCCESS;
}

extern "C" int lagr_wait(lagr_ctx ctx, char *msg)
{
    if (!ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    flush_deferred(ctx);
    return lagr_ok(msg);
}

// ----------------------------------------------------------- kernel timing

static void timers_clear(lagr_ctx ctx)
{
    for (auto &t : ctx->timers) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    ctx->timers.clear();
}

void timer_begin(lagr_ctx ctx, const char *name, hipEvent_t *stop)
{
    KernelTimer t;
    t.name = name;
    if (hipEventCreate(&t.start) != hipSuccess) return;
    if (hipEventCreate(&t.stop) != hipSuccess) {
        (void)hipEventDestroy(t.start);
        return;
    }
    (void)hipEventRecord(t.start, ctx->stream);
    *stop = t.stop;
    ctx->timers.push_back(t);
}

void timer_end(lagr_ctx ctx, hipEvent_t stop) { (void)hipEventRecord(stop, ctx->stream); }

extern "C" int lagr_ctx_timing(lagr_ctx ctx, int enable, char *msg)
{
    if (!ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    timers_clear(ctx);
    ctx->timing = enable ? 1 : 0;
    return lagr_ok(msg);
}

extern "C" int lagr_ctx_kernel_time(lagr_ctx ctx, const char *kernel, double *total_ms,
                                    int64_t *launches, char *msg)
{
    if (!ctx || !kernel) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &t : ctx->timers) {
        if (t.name != kernel) continue;
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, t.start, t.stop));
        tot += ms;
        cnt++;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return lagr_ok(msg);
}

void *ws_get(lagr_ctx ctx, WsSlot slot, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (ctx->ws_bytes[slot] >= bytes) return ctx->ws[slot];
    if (ctx->ws[slot]) {
        // queued work may still read the old buffer
        (void)hipStreamSynchronize(ctx->stream);
        flush_deferred(ctx);
        dev_free(ctx->ws[slot], ctx->ws_bytes[slot]);
        ctx->ws[slot] = nullptr;
        ctx->ws_bytes[slot] = 0;
    }
    size_t grow = bytes + bytes / 8;
    grow = (grow + 255) & ~(size_t)255;
    void *p = dev_alloc(grow);
    if (!p) return nullptr;
    ctx->ws[slot] = p;
    ctx->ws_bytes[slot] = grow;
    return p;
}

// ------------------------------------------------------------- matrices

void defer_free(lagr_ctx ctx, void *p, size_t bytes)
{
    if (!p) return;
    ctx->deferred.emplace_back(p, bytes);
    ctx->deferred_bytes += bytes;
    if (ctx->deferred_bytes > ((size_t)2 << 30)) {
        (void)hipStreamSynchronize(ctx->stream);
        flush_deferred(ctx);
    }
}

size_t ctx_retained_bytes(const lagr_ctx ctx)
{
    size_t b = ctx->lv_bytes * ctx->lvpool.size() + ctx->vspare_pb + ctx->vspare_vb + ctx->deferred_bytes;
    for (int s = 0; s < WS_NSLOTS; s++) b += ctx->ws_bytes[s];
    return b;
}

void ctx_trim(lagr_ctx ctx)
{
    (void)hipStreamSynchronize(ctx->stream);
    flush_deferred(ctx);
    // captured graphs point into the workspace: drop them with it
    if (ctx->bfs_exec) (void)hipGraphExecDestroy(ctx->bfs_exec);
    if (ctx->bfs_exec_more) (void)hipGraphExecDestroy(ctx->bfs_exec_more);
    if (ctx->bfs_graph) (void)hipGraphDestroy(ctx->bfs_graph);
    if (ctx->sssp_exec) (void)hipGraphExecDestroy(ctx->sssp_exec);
    if (ctx->ms_exec) (void)hipGraphExecDestroy(ctx->ms_exec);
    ctx->bfs_exec = ctx->bfs_exec_more = nullptr;
    ctx->bfs_graph = nullptr;
    ctx->bfs_start_node = nullptr;
    ctx->bfs_key = -1;
    ctx->bfs_state = nullptr;
    ctx->bfs_ctr = nullptr;
    ctx->sssp_exec = nullptr;
    ctx->sssp_key = -1;
    ctx->sssp_state = nullptr;
    ctx->ms_exec = nullptr;
    ctx->ms_key.clear();
    for (int s = 0; s < WS_NSLOTS; s++) {
        dev_free(ctx->ws[s], ctx->ws_bytes[s]);
        ctx->ws[s] = nullptr;
        ctx->ws_bytes[s] = 0;
    }
    for (void *p : ctx->lvpool) dev_free(p, ctx->lv_bytes);
    ctx->lvpool.clear();
    dev_free(ctx->vspare_present, ctx->vspare_pb);
    dev_free(ctx->vspare_values, ctx->vspare_vb);
    ctx->vspare_present = nullptr;
    ctx->vspare_values = nullptr;
    ctx->vspare_pb = ctx->vspare_vb = 0;
    ctx->vxm_cand = nullptr;
    ctx->vxm_cand_n = 0;
}

void flush_deferred(lagr_ctx ctx)
{
    for (auto &b : ctx->deferred) dev_free(b.first, b.second);
    ctx->deferred.clear();
    ctx->deferred_bytes = 0;
}

void matrix_release_arrays_later(lagr_ctx ctx, lagr_matrix A)
{
    if (A->tcache) {
        matrix_release_arrays_later(ctx, A->tcache);
        delete A->tcache;
        A->tcache = nullptr;
    }
    if (A->rowptr_bytes) defer_free(ctx, A->rowptr, A->rowptr_bytes);
    if (A->colidx_bytes) defer_free(ctx, A->colidx, A->colidx_bytes);
    if (A->values_bytes) defer_free(ctx, A->values, A->values_bytes);
    A->rowptr = nullptr;
    A->colidx = nullptr;
    A->values = nullptr;
    A->rowptr_bytes = A->colidx_bytes = A->values_bytes = 0;
}

void vector_release_arrays_later(lagr_ctx ctx, lagr_vector v)
{
    if (v->idx_bytes) defer_free(ctx, v->idx, v->idx_bytes);
    if (v->present_bytes) defer_free(ctx, v->present, v->present_bytes);
    if (v->values_bytes) defer_free(ctx, v->values, v->values_bytes);
    v->idx = nullptr;
    v->present = nullptr;
    v->values = nullptr;
    v->idx_bytes = v->present_bytes = v->values_bytes = 0;
    v->nvals = 0;
    v->count_dev = nullptr;
}

void matrix_release_arrays(lagr_matrix A)
{
    if (A->tcache) lagr_matrix_free(&A->tcache);
    if (A->rowptr_bytes) dev_free(A->rowptr, A->rowptr_bytes);
    if (A->colidx_bytes) dev_free(A->colidx, A->colidx_bytes);
    if (A->values_bytes) dev_free(A->values, A->values_bytes);
    A->rowptr = nullptr;
    A->colidx = nullptr;
    A->values = nullptr;
    A->rowptr_bytes = A->colidx_bytes = A->values_bytes = 0;
    A->nvals = 0;
}

int matrix_alloc(lagr_matrix A, int64_t nvals, char *msg)
{
    size_t rb = sizeof(int64_t) * (size_t)(A->nrows + 1);
    size_t cb = sizeof(int32_t) * (size_t)(nvals > 0 ? nvals : 1);
    size_t vb = type_size(A->type) * (size_t)(nvals > 0 ? nvals : 1);
    int64_t *rp = (int64_t *)dev_alloc(rb);
    int32_t *ci = (int32_t *)dev_alloc(cb);
    void *va = vb ? dev_alloc(vb) : nullptr;
    if (!rp || !ci || (vb && !va)) {
        dev_free(rp, rb);
        dev_free(ci, cb);
        dev_free(va, vb);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix arrays (%lld entries)", (long long)nvals);
    }
    A->rowptr = rp;
    A->colidx = ci;
    A->values = va;
    A->rowptr_bytes = rb;
    A->colidx_bytes = cb;
    A->values_bytes = vb;
    A->nvals = nvals;
    return LAGR_SUCCESS;
}

static int check_type(lagr_type t, char *msg)
{
    if (t != LAGR_BOOL && t != LAGR_INT64 && t != LAGR_FP64 && t != LAGR_INT32)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown type %d", (int)t);
    return LAGR_SUCCESS;
}

namespace {
__global__ void k_widen_i32(const int32_t *__restrict__ s, int64_t *__restrict__ d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}
__global__ void k_narrow_i64(const int64_t *__restrict__ s, int32_t *__restrict__ d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (int32_t)s[i];
}

// A library-owned widened copy of n int32 values (nullptr on failure).
int64_t *widened_copy(lagr_ctx ctx, const void *values, int64_t n, size_t *bytes, char *msg)
{
    *bytes = 8 * (size_t)(n > 0 ? n : 1);
    int64_t *w = (int64_t *)dev_alloc(*bytes);
    if (!w) {
        lagr_fail(msg, LAGR_OUT_OF_MEMORY, "INT32 values");
        return nullptr;
    }
    if (widen_i32(ctx, (const int32_t *)values, w, n, msg) < 0) {
        dev_free(w, *bytes);
        return nullptr;
    }
    return w;
}
}  // namespace

int widen_i32(lagr_ctx ctx, const int32_t *src, int64_t *dst, int64_t n, char *msg)
{
    if (n <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_widen_i32, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream, src, dst, n);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

int narrow_i64(lagr_ctx ctx, const int64_t *src, int32_t *dst, int64_t n, char *msg)
{
    if (n <= 0) return LAGR_SUCCESS;
    hipLaunchKernelGGL(k_narrow_i64, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream, src, dst, n);
    LAUNCH_CHECK();
    return LAGR_SUCCESS;
}

extern "C" int lagr_matrix_new(lagr_matrix *A, lagr_type type, int64_t nrows, int64_t ncols,
                               lagr_ctx ctx, char *msg)
{
    if (!A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *A = nullptr;
    TRY(check_type(type, msg));
    if (nrows < 0 || ncols < 0 || nrows > INT32_MAX || ncols > INT32_MAX)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "dimensions %lld x %lld out of range",
                         (long long)nrows, (long long)ncols);
    lagr_matrix M = new (std::nothrow) lagr_matrix_s();
    if (!M) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    M->type = type;
    M->nrows = nrows;
    M->ncols = ncols;
    int rc = matrix_alloc(M, 0, msg);
    if (rc < 0) {
        delete M;
        return rc;
    }
    rc = fill_i64(ctx, M->rowptr, nrows + 1, 0, msg);
    if (rc < 0) {
        matrix_release_arrays(M);
        delete M;
        return rc;
    }
    *A = M;
    return lagr_ok(msg);
}

extern "C" int lagr_matrix_wrap_csr(lagr_matrix *A, lagr_type type, int64_t nrows, int64_t ncols,
                                    int64_t nvals, const int64_t *rowptr, const int32_t *colidx,
                                    const void *values, lagr_ctx ctx, char *msg)
{
    if (!A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *A = nullptr;
    TRY(check_type(type, msg));
    if (nrows < 0 || ncols < 0 || nrows > INT32_MAX || ncols > INT32_MAX || nvals < 0)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "bad sizes");
    if (!rowptr) return lagr_fail(msg, LAGR_NULL_POINTER, "rowptr is NULL");
    if (nvals > 0 && !colidx) return lagr_fail(msg, LAGR_NULL_POINTER, "colidx is NULL");
    if (type != LAGR_BOOL && nvals > 0 && !values)
        return lagr_fail(msg, LAGR_NULL_POINTER, "values are NULL for a valued type");
    lagr_matrix M = new (std::nothrow) lagr_matrix_s();
    if (!M) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    M->type = type;
    M->nrows = nrows;
    M->ncols = ncols;
    M->nvals = nvals;
    M->rowptr = const_cast<int64_t *>(rowptr);
    M->colidx = const_cast<int32_t *>(colidx);
    M->values = type == LAGR_BOOL ? nullptr : const_cast<void *>(values);
    if (type == LAGR_INT32) {
        M->values = widened_copy(ctx, values, nvals, &M->values_bytes, msg);
        if (!M->values) {
            delete M;
            return LAGR_OUT_OF_MEMORY;
        }
    }
    *A = M;
    return lagr_ok(msg);
}

extern "C" int lagr_matrix_info(const lagr_matrix A, lagr_type *type, int64_t *nrows,
                                int64_t *ncols, int64_t *nvals, char *msg)
{
    if (!A) return lagr_fail(msg, LAGR_NULL_POINTER, "matrix is NULL");
    if (type) *type = A->type;
    if (nrows) *nrows = A->nrows;
    if (ncols) *ncols = A->ncols;
    if (nvals) *nvals = A->nvals;
    return lagr_ok(msg);
}

extern "C" int lagr_matrix_nvals(int64_t *nvals, const lagr_matrix A, lagr_ctx ctx, char *msg)
{
    if (!A || !nvals) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *nvals = A->nvals;
    return lagr_ok(msg);
}

extern "C" int lagr_matrix_extract_csr(const lagr_matrix A, int64_t *rowptr, int32_t *colidx,
                                       void *values, lagr_ctx ctx, char *msg)
{
    if (!A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (rowptr)
        HIP_TRY(hipMemcpyAsync(rowptr, A->rowptr, sizeof(int64_t) * (A->nrows + 1),
                               hipMemcpyDeviceToDevice, ctx->stream));
    if (colidx && A->nvals)
        HIP_TRY(hipMemcpyAsync(colidx, A->colidx, sizeof(int32_t) * A->nvals,
                               hipMemcpyDeviceToDevice, ctx->stream));
    if (values && A->nvals && A->type == LAGR_INT32)
        TRY(narrow_i64(ctx, (const int64_t *)A->values, (int32_t *)values, A->nvals, msg));
    else if (values && A->nvals && A->type != LAGR_BOOL)
        HIP_TRY(hipMemcpyAsync(values, A->values, 8 * A->nvals, hipMemcpyDeviceToDevice,
                               ctx->stream));
    return lagr_ok(msg);
}

extern "C" int lagr_matrix_free(lagr_matrix *A)
{
    if (!A || !*A) return LAGR_SUCCESS;
    matrix_release_arrays(*A);
    delete *A;
    *A = nullptr;
    return LAGR_SUCCESS;
}

// --------------------------------------------------------------- vectors

void vector_release_arrays(lagr_vector v)
{
    if (v->idx_bytes) dev_free(v->idx, v->idx_bytes);
    if (v->present_bytes) dev_free(v->present, v->present_bytes);
    if (v->values_bytes) dev_free(v->values, v->values_bytes);
    v->idx = nullptr;
    v->present = nullptr;
    v->values = nullptr;
    v->idx_bytes = v->present_bytes = v->values_bytes = 0;
    v->nvals = 0;
    v->count_dev = nullptr;
}

extern "C" int lagr_vector_new(lagr_vector *v, lagr_type type, int64_t n, lagr_ctx ctx, char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *v = nullptr;
    TRY(check_type(type, msg));
    if (n < 0 || n > INT32_MAX) return lagr_fail(msg, LAGR_INVALID_VALUE, "bad length");
    lagr_vector x = new (std::nothrow) lagr_vector_s();
    if (!x) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    x->type = type;
    x->n = n;
    x->fmt = LAGR_VEC_SPARSE;
    x->nvals = 0;
    *v = x;
    return lagr_ok(msg);
}

extern "C" int lagr_vector_wrap_sparse(lagr_vector *v, lagr_type type, int64_t n, int64_t nvals,
                                       const int32_t *idx, const void *values, lagr_ctx ctx,
                                       char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *v = nullptr;
    TRY(check_type(type, msg));
    if (n < 0 || n > INT32_MAX || nvals < 0 || nvals > n)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "bad sizes");
    if (nvals > 0 && !idx) return lagr_fail(msg, LAGR_NULL_POINTER, "idx is NULL");
    if (type != LAGR_BOOL && nvals > 0 && !values)
        return lagr_fail(msg, LAGR_NULL_POINTER, "values are NULL for a valued type");
    lagr_vector x = new (std::nothrow) lagr_vector_s();
    if (!x) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    x->type = type;
    x->n = n;
    x->fmt = LAGR_VEC_SPARSE;
    x->nvals = nvals;
    x->idx = const_cast<int32_t *>(idx);
    x->values = type == LAGR_BOOL ? nullptr : const_cast<void *>(values);
    if (type == LAGR_INT32 && !(x->values = widened_copy(ctx, values, nvals, &x->values_bytes, msg))) {
        delete x;
        return LAGR_OUT_OF_MEMORY;
    }
    *v = x;
    return lagr_ok(msg);
}

extern "C" int lagr_vector_wrap_bitmap(lagr_vector *v, lagr_type type, int64_t n,
                                       const uint8_t *present, const void *values, lagr_ctx ctx,
                                       char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *v = nullptr;
    TRY(check_type(type, msg));
    if (n < 0 || n > INT32_MAX) return lagr_fail(msg, LAGR_INVALID_VALUE, "bad length");
    if (n > 0 && !present) return lagr_fail(msg, LAGR_NULL_POINTER, "present is NULL");
    if (type != LAGR_BOOL && n > 0 && !values)
        return lagr_fail(msg, LAGR_NULL_POINTER, "values are NULL for a valued type");
    lagr_vector x = new (std::nothrow) lagr_vector_s();
    if (!x) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    x->type = type;
    x->n = n;
    x->fmt = LAGR_VEC_BITMAP;
    x->nvals = -1;
    x->present = const_cast<uint8_t *>(present);
    x->values = type == LAGR_BOOL ? nullptr : const_cast<void *>(values);
    if (type == LAGR_INT32 && !(x->values = widened_copy(ctx, values, n, &x->values_bytes, msg))) {
        delete x;
        return LAGR_OUT_OF_MEMORY;
    }
    *v = x;
    return lagr_ok(msg);
}

extern "C" int lagr_vector_wrap_full(lagr_vector *v, lagr_type type, int64_t n, const void *values,
                                     lagr_ctx ctx, char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    *v = nullptr;
    TRY(check_type(type, msg));
    if (type == LAGR_BOOL) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "a FULL vector needs values");
    if (n < 0 || n > INT32_MAX) return lagr_fail(msg, LAGR_INVALID_VALUE, "bad length");
    if (n > 0 && !values) return lagr_fail(msg, LAGR_NULL_POINTER, "values are NULL");
    lagr_vector x = new (std::nothrow) lagr_vector_s();
    if (!x) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector");
    x->type = type;
    x->n = n;
    x->fmt = LAGR_VEC_FULL;
    x->nvals = n;
    x->values = const_cast<void *>(values);
    if (type == LAGR_INT32 && !(x->values = widened_copy(ctx, values, n, &x->values_bytes, msg))) {
        delete x;
        return LAGR_OUT_OF_MEMORY;
    }
    *v = x;
    return lagr_ok(msg);
}

extern "C" int lagr_vector_info(const lagr_vector v, lagr_type *type, int64_t *n,
                                lagr_vformat *format, char *msg)
{
    if (!v) return lagr_fail(msg, LAGR_NULL_POINTER, "vector is NULL");
    if (type) *type = v->type;
    if (n) *n = v->n;
    if (format) *format = v->fmt;
    return lagr_ok(msg);
}

extern "C" int lagr_vector_free(lagr_vector *v)
{
    if (!v || !*v) return LAGR_SUCCESS;
    vector_release_arrays(*v);
    delete *v;
    *v = nullptr;
    return LAGR_SUCCESS;
}
