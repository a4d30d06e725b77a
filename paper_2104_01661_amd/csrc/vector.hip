// Vector queries and conversions between the SPARSE, BITMAP and FULL
// storage (the list and bitmap forms of a frontier, Section VI-A).
#include "internal.h"

namespace {

__global__ void k_present_flags(const uint8_t *__restrict__ present, int64_t n,
                                int64_t *__restrict__ flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = present[i] ? 1 : 0;
}

__global__ void k_compact_bitmap(const uint8_t *__restrict__ present, const uint64_t *__restrict__ vals,
                                 int64_t n, const int64_t *__restrict__ pos, int32_t *__restrict__ idx,
                                 uint64_t *__restrict__ ovals)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!present[i]) continue;
        const int64_t q = pos[i];
        if (idx) idx[q] = (int32_t)i;
        if (ovals) ovals[q] = vals[i];
    }
}

__global__ void k_iota_i32(int32_t *__restrict__ idx, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = (int32_t)i;
}

__global__ void k_dense_from_sparse(const int32_t *__restrict__ idx, const uint64_t *__restrict__ vals,
                                    int64_t nvals, uint8_t *__restrict__ present,
                                    uint64_t *__restrict__ ovals)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nvals;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (present) present[idx[q]] = 1;
        if (ovals && vals) ovals[idx[q]] = vals[q];
    }
}

__global__ void k_dense_from_bitmap(const uint8_t *__restrict__ pin, const uint64_t *__restrict__ vin,
                                    int64_t n, uint64_t fill, uint8_t *__restrict__ pout,
                                    uint64_t *__restrict__ vout)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t p = pin ? pin[i] : 1;
        if (pout) pout[i] = p;
        if (vout) vout[i] = (p && vin) ? vin[i] : fill;
    }
}

}  // namespace

// Number of entries of a bitmap vector (synchronises).
int bitmap_count(lagr_ctx ctx, const uint8_t *present, int64_t n, int64_t *count, char *msg)
{
    int64_t *flags = (int64_t *)ws_get(ctx, WS_GEN_H, sizeof(int64_t) * (n > 0 ? n : 1));
    if (!flags) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "nvals workspace");
    if (n > 0) {
        hipLaunchKernelGGL(k_present_flags, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                           present, n, flags);
        LAUNCH_CHECK();
    }
    return scan_exclusive_i64(ctx, flags, flags, n, count, msg);
}

// Sorted tuples of any vector into caller buffers (idx / vals may be NULL).
// For a BITMAP vector, *nvals receives the count.
int vector_tuples(lagr_ctx ctx, const lagr_vector v, int32_t *idx, void *vals, int64_t *nvals,
                  char *msg)
{
    const bool valued = v->type != LAGR_BOOL;
    if (v->fmt == LAGR_VEC_SPARSE) {
        if (nvals) *nvals = v->nvals;
        if (idx && v->nvals)
            HIP_TRY(hipMemcpyAsync(idx, v->idx, sizeof(int32_t) * v->nvals, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        if (vals && valued && v->nvals)
            HIP_TRY(hipMemcpyAsync(vals, v->values, 8 * v->nvals, hipMemcpyDeviceToDevice, ctx->stream));
        return LAGR_SUCCESS;
    }
    if (v->fmt == LAGR_VEC_FULL) {
        if (nvals) *nvals = v->n;
        if (idx && v->n) {
            hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(v->n, 256, 16384)), dim3(256), 0, ctx->stream,
                               idx, v->n);
            LAUNCH_CHECK();
        }
        if (vals && v->n)
            HIP_TRY(hipMemcpyAsync(vals, v->values, 8 * v->n, hipMemcpyDeviceToDevice, ctx->stream));
        return LAGR_SUCCESS;
    }
    const int64_t n = v->n;
    int64_t *pos = (int64_t *)ws_get(ctx, WS_GEN_H, sizeof(int64_t) * (n > 0 ? n : 1));
    if (!pos) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "tuples workspace");
    int64_t cnt = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_present_flags, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                           v->present, n, pos);
        LAUNCH_CHECK();
    }
    TRY(scan_exclusive_i64(ctx, pos, pos, n, &cnt, msg));
    if (nvals) *nvals = cnt;
    if (n > 0 && (idx || vals)) {
        hipLaunchKernelGGL(k_compact_bitmap, dim3(grid_for(n, 256, 16384)), dim3(256), 0, ctx->stream,
                           v->present, (const uint64_t *)v->values, n, pos, idx,
                           valued ? (uint64_t *)vals : nullptr);
        LAUNCH_CHECK();
    }
    return LAGR_SUCCESS;
}

extern "C" int lagr_vector_nvals(int64_t *nvals, const lagr_vector v, lagr_ctx ctx, char *msg)
{
    if (!nvals || !v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (v->fmt == LAGR_VEC_BITMAP && v->count_dev) {
        unsigned long long c = 0;
        TRY(read_back(ctx, &c, v->count_dev, sizeof(c), msg));
        *nvals = (int64_t)c;
    } else if (v->fmt == LAGR_VEC_BITMAP) {
        TRY(bitmap_count(ctx, v->present, v->n, nvals, msg));
    } else {
        *nvals = v->nvals;
    }
    return lagr_ok(msg);
}

extern "C" int lagr_vector_extract_tuples(const lagr_vector v, int32_t *idx, void *values,
                                          lagr_ctx ctx, char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    int64_t nv = 0;
    if (v->type == LAGR_INT32 && values) {
        // the values go through 8-byte slots, then narrow
        TRY(lagr_vector_nvals(&nv, v, ctx, msg));
        int64_t *tmp = (int64_t *)ws_get(ctx, WS_GEN_G, 8 * (size_t)(nv > 0 ? nv : 1));
        if (!tmp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "extract");
        TRY(vector_tuples(ctx, v, idx, tmp, &nv, msg));
        TRY(narrow_i64(ctx, tmp, (int32_t *)values, nv, msg));
        return lagr_ok(msg);
    }
    TRY(vector_tuples(ctx, v, idx, values, &nv, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_vector_extract_dense(const lagr_vector v, uint8_t *present, void *values,
                                         const void *fill, lagr_ctx ctx, char *msg)
{
    if (!v || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    const int64_t n = v->n;
    uint64_t f = 0;
    if (fill && v->type == LAGR_INT32) {
        int32_t f32;
        memcpy(&f32, fill, 4);
        f = (uint64_t)(int64_t)f32;
    } else if (fill && v->type != LAGR_BOOL) {
        memcpy(&f, fill, 8);
    }
    if (v->type == LAGR_BOOL) values = nullptr;
    if (n == 0) return lagr_ok(msg);
    void *out32 = nullptr;      // INT32: the caller's array, filled by narrowing
    if (v->type == LAGR_INT32 && values) {
        out32 = values;
        values = ws_get(ctx, WS_GEN_G, 8 * (size_t)n);
        if (!values) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "extract");
    }
    if (v->fmt == LAGR_VEC_SPARSE) {
        hipLaunchKernelGGL(k_dense_from_bitmap, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                           ctx->stream, (const uint8_t *)nullptr, (const uint64_t *)nullptr, n, f,
                           (uint8_t *)nullptr, (uint64_t *)values);
        LAUNCH_CHECK();
        if (present) TRY(fill_u8(ctx, present, n, 0, msg));
        if (v->nvals) {
            hipLaunchKernelGGL(k_dense_from_sparse, dim3(grid_for(v->nvals, 256, 16384)), dim3(256), 0,
                               ctx->stream, v->idx, (const uint64_t *)v->values, v->nvals, present,
                               (uint64_t *)values);
            LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL(k_dense_from_bitmap, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                           ctx->stream, v->fmt == LAGR_VEC_BITMAP ? v->present : nullptr,
                           (const uint64_t *)v->values, n, f, present, (uint64_t *)values);
        LAUNCH_CHECK();
    }
    if (out32) TRY(narrow_i64(ctx, (const int64_t *)values, (int32_t *)out32, n, msg));
    return lagr_ok(msg);
}
