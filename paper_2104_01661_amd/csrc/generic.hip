// Generic masked semiring operations on CSR matrices and vectors (Section
// III: Table I operations, Table II semirings, "Masks"):
//   mxm / vxm          C<M> accum= A' (+).(x) B'
//   eWiseAdd / Mult     C<M> accum= A op B on the union / intersection
//   assign              w<m>(:) accum= u,  w<m>(:) accum= s
//   reduce              rows of A' to a vector, everything to a scalar
//
// Every operation computes an unmasked-by-rule result T, then one merge per
// row applies the mask, the accumulator and replace to the old C.  Vectors
// are handled as 1 x n matrices.  The products come in two forms:
//   * dot form, when a mask is present and not complemented: each mask
//     entry (i, j) intersects the sorted rows A'_i and (B'^T)_j, one thread
//     per entry, combining in ascending k (plus.pair uses the wavefront
//     kernel of tc_device.h);
//   * saxpy form otherwise (Gustavson): every product A'(i,k) B'(k,j) is
//     written out, sorted stably by (i, j), and each run is combined in
//     ascending k.  `any` keeps the first, i.e. the smallest k.
// Transposed inputs are transposed explicitly.  All temporaries are
// allocated per call and the call waits for the stream before it returns.
#include <mutex>
#include <new>

#include "internal.h"
#include "tc_device.h"

int vector_tuples(lagr_ctx ctx, const lagr_vector v, int32_t *idx, void *vals, int64_t *nvals,
                  char *msg);

namespace {

// ------------------------------------------------------------ value algebra

// Values travel as 64-bit words holding an int64, a double or a
// sign-extended int32 (whose arithmetic wraps modulo 2^32).
enum VKind { VK_I64 = 0, VK_F64 = 1, VK_I32 = 2 };

__device__ __forceinline__ uint64_t wrap32(int64_t x) { return (uint64_t)(int64_t)(int32_t)(uint32_t)x; }

__host__ __device__ __forceinline__ double bits_f(uint64_t b)
{
    double d;
    memcpy(&d, &b, 8);
    return d;
}
__host__ __device__ __forceinline__ uint64_t f_bits(double d)
{
    uint64_t b;
    memcpy(&b, &d, 8);
    return b;
}

// value of entry p of a CSR with optional values (BOOL: 1)
__device__ __forceinline__ uint64_t load_val(const uint64_t *val, int64_t p, int vk)
{
    if (val) return val[p];
    return vk == VK_F64 ? f_bits(1.0) : (uint64_t)1;
}

// convert a stored value of kind `from` to kind `to`
__device__ __forceinline__ uint64_t convert(uint64_t x, int from, int to)
{
    if (from == to) return x;
    if (to == VK_F64) return f_bits((double)(int64_t)x);
    const uint64_t i = from == VK_F64 ? (uint64_t)(int64_t)bits_f(x) : x;
    return to == VK_I32 ? wrap32((int64_t)i) : i;
}

__device__ __forceinline__ uint64_t binop(int op, int vk, uint64_t c, uint64_t t)
{
    if (vk == VK_F64) {
        const double x = bits_f(c), y = bits_f(t);
        switch (op) {
        case LAGR_PLUS: return f_bits(x + y);
        case LAGR_MIN: return f_bits(y < x ? y : x);
        case LAGR_FIRST:
        case LAGR_ANY: return c;
        case LAGR_SECOND: return t;
        case LAGR_TIMES: return f_bits(x * y);
        case LAGR_DIV: return f_bits(x / y);
        default: return t;
        }
    }
    const int64_t x = (int64_t)c, y = (int64_t)t;
    uint64_t r;
    switch (op) {
    case LAGR_PLUS: r = (uint64_t)x + (uint64_t)y; break;
    case LAGR_MIN: r = (uint64_t)(y < x ? y : x); break;
    case LAGR_FIRST:
    case LAGR_ANY: r = c; break;
    case LAGR_SECOND: r = t; break;
    case LAGR_TIMES: r = (uint64_t)x * (uint64_t)y; break;
    default: r = t; break;
    }
    return vk == VK_I32 ? wrap32((int64_t)r) : r;
}

struct Sem {
    int semiring;
    int astore;  // kind A' values are stored as
    int bstore;
    int akind;   // kind the semiring reads them as
    int bkind;
    int okind;   // result kind
};

__device__ __forceinline__ uint64_t load_a(const Sem &s, const uint64_t *val, int64_t p)
{
    return convert(load_val(val, p, s.astore), s.astore, s.akind);
}
__device__ __forceinline__ uint64_t load_b(const Sem &s, const uint64_t *val, int64_t p)
{
    return convert(load_val(val, p, s.bstore), s.bstore, s.bkind);
}

// one product term A'(i,k) (x) B'(k,j)
__device__ __forceinline__ uint64_t sem_mult(const Sem &s, uint64_t a, uint64_t b, int64_t k)
{
    switch (s.semiring) {
    case LAGR_PLUS_PAIR: return 1;
    case LAGR_ANY_SECONDI: return (uint64_t)k;
    case LAGR_PLUS_FIRST: return a;
    default: return f_bits(bits_f(a) + bits_f(b));   // MIN_PLUS, FP64
    }
}

// accumulate term t into r (ascending k order; any keeps the first)
__device__ __forceinline__ uint64_t sem_add(const Sem &s, uint64_t r, uint64_t t)
{
    switch (s.semiring) {
    case LAGR_PLUS_PAIR: return r + t;
    case LAGR_ANY_SECONDI: return r;
    case LAGR_PLUS_FIRST:
        return s.okind == VK_F64 ? f_bits(bits_f(r) + bits_f(t)) : s.okind == VK_I32 ? wrap32((int64_t)(r + t)) : r + t;
    default: {
        const double x = bits_f(r), y = bits_f(t);
        return f_bits(y < x ? y : x);
    }
    }
}

// --------------------------------------------------------------- CSR view

struct Csr {
    int64_t nrows = 0, ncols = 0, nvals = 0;
    const int64_t *rp = nullptr;
    const int32_t *ci = nullptr;
    const uint64_t *val = nullptr;
    lagr_type type = LAGR_BOOL;
};

// Value of a valued mask entry as a truth value (Section III, "Masks": an
// entry that is present and nonzero).  For FP64 both +0.0 and -0.0 are zero,
// so the sign bit is ignored; any other bit pattern (NaN included) is true.
__device__ __forceinline__ bool mask_value_true(const Csr &M, int64_t p)
{
    const uint64_t b = M.val[p];
    return M.type == LAGR_FP64 ? (b << 1) != 0 : b != 0;
}

__global__ void k_iota32(int32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_two(int64_t *__restrict__ rp, int64_t a, int64_t b)
{
    rp[0] = a;
    rp[1] = b;
}

// row of each entry by binary search of the row offsets
__device__ __forceinline__ int64_t row_of(const int64_t *rp, int64_t nrows, int64_t p)
{
    int64_t lo = 0, hi = nrows;   // last r with rp[r] <= p
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_tr_keys(const Csr A, int ebits, uint64_t *__restrict__ keys)
{
    const int64_t nrows = A.nrows;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.nvals;
         p += (int64_t)gridDim.x * blockDim.x)
        keys[p] = ((uint64_t)A.ci[p] << ebits) | (uint64_t)p;
    (void)nrows;
}

__global__ void k_tr_fill(const Csr A, const uint64_t *__restrict__ keys, int ebits,
                          int32_t *__restrict__ ci, uint64_t *__restrict__ val)
{
    const uint64_t emask = (ebits >= 64) ? ~0ull : ((1ull << ebits) - 1);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < A.nvals;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = (int64_t)(keys[q] & emask);
        ci[q] = (int32_t)row_of(A.rp, A.nrows, p);
        if (val) val[q] = A.val[p];
    }
}

// ------------------------------------------------------------ dot form

__global__ void k_dot(const Csr M, const Csr A, const Csr BT, int valued_mask, Sem s,
                      uint64_t *__restrict__ out, uint8_t *__restrict__ has)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M.nvals;
         q += (int64_t)gridDim.x * blockDim.x) {
        has[q] = 0;
        if (valued_mask && M.val && !mask_value_true(M, q)) continue;   // explicit zero
        const int64_t i = row_of(M.rp, M.nrows, q);
        const int64_t j = M.ci[q];
        int64_t a = A.rp[i], ae = A.rp[i + 1], b = BT.rp[j], be = BT.rp[j + 1];
        bool any = false;
        uint64_t r = 0;
        while (a < ae && b < be) {
            const int32_t ka = A.ci[a], kb = BT.ci[b];
            if (ka < kb) a++;
            else if (ka > kb) b++;
            else {
                const uint64_t t = sem_mult(s, load_a(s, A.val, a), load_b(s, BT.val, b), ka);
                r = any ? sem_add(s, r, t) : t;
                any = true;
                a++;
                b++;
            }
        }
        if (any) {
            out[q] = r;
            has[q] = 1;
        }
    }
}

__global__ void k_counts_to_has(const int64_t *__restrict__ cnt, int64_t n, const Csr M, int valued_mask,
                                uint64_t *__restrict__ out, uint8_t *__restrict__ has)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const bool masked_out = valued_mask && M.val && !mask_value_true(M, q);
        has[q] = (!masked_out && cnt[q] > 0) ? 1 : 0;
        out[q] = (uint64_t)cnt[q];
    }
}

// compaction of flagged entries (rows keep their order)
__global__ void k_flags_i64(const uint8_t *__restrict__ has, int64_t n, int64_t *__restrict__ f)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        f[q] = has[q] ? 1 : 0;
}

__global__ void k_compact(const Csr M, const uint8_t *__restrict__ has, const int64_t *__restrict__ pos,
                          const uint64_t *__restrict__ vin, int32_t *__restrict__ ci,
                          uint64_t *__restrict__ vout)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M.nvals;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (!has[q]) continue;
        ci[pos[q]] = M.ci[q];
        if (vout) vout[pos[q]] = vin[q];
    }
}

__global__ void k_rowptr_compacted(const Csr M, const int64_t *__restrict__ pos, int64_t total,
                                   int64_t *__restrict__ rp)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= M.nrows;
         r += (int64_t)gridDim.x * blockDim.x)
        rp[r] = pos[M.rp[r]];
}

// ----------------------------------------------------------- saxpy form

__global__ void k_flops(const Csr A, const Csr B, int64_t *__restrict__ fl)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t f = 0;
        for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++) {
            const int32_t k = A.ci[p];
            f += B.rp[k + 1] - B.rp[k];
        }
        fl[i] = f;
    }
}

// products in (k ascending, then B'_k order) per row; keys carry (row, col,
// product index) so a sort keeps equal (row, col) runs in k order
__global__ void k_expand(const Csr A, const Csr B, const int64_t *__restrict__ off, Sem s,
                         int cbits, int fbits, uint64_t *__restrict__ keys, uint64_t *__restrict__ vals)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = off[i];
        for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++) {
            const int32_t k = A.ci[p];
            const uint64_t av = load_a(s, A.val, p);
            for (int64_t q = B.rp[k]; q < B.rp[k + 1]; q++) {
                const int32_t j = B.ci[q];
                keys[o] = (((uint64_t)i << cbits | (uint64_t)j) << fbits) | (uint64_t)o;
                vals[o] = sem_mult(s, av, load_b(s, B.val, q), k);
                o++;
            }
        }
    }
}

// mask test at (i, j): M row i is sorted; binary search
__device__ __forceinline__ bool mask_at(const Csr &M, bool has_mask, bool structural, bool comp,
                                        int64_t i, int32_t j)
{
    bool on = true;
    if (has_mask) {
        int64_t lo = M.rp[i], hi = M.rp[i + 1];
        const int64_t end = hi;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (M.ci[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        on = lo < end && M.ci[lo] == j;
        if (on && !structural && M.val) on = mask_value_true(M, lo);
    }
    return comp ? !on : on;
}

// run heads of the sorted products; products the (complemented) mask
// discards are dropped here (they could never be written)
__global__ void k_run_heads(const uint64_t *__restrict__ keys, int64_t F, int fbits, int cbits,
                            const Csr M, int has_mask, int structural, int comp,
                            int64_t *__restrict__ head)
{
    const uint64_t cm = (1ull << cbits) - 1;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < F;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t rc = keys[q] >> fbits;
        const bool first = q == 0 || (keys[q - 1] >> fbits) != rc;
        bool keep = first;
        if (keep && (has_mask || comp))
            keep = mask_at(M, has_mask, structural, comp, (int64_t)(rc >> cbits), (int32_t)(rc & cm));
        head[q] = keep ? 1 : 0;
    }
}

__global__ void k_runs_reduce(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ vals,
                              int64_t F, int fbits, int cbits, const int64_t *__restrict__ pos,
                              const int64_t *__restrict__ headflag, Sem s, int32_t *__restrict__ ci,
                              uint64_t *__restrict__ vout, uint64_t *__restrict__ rows_key)
{
    const uint64_t cm = (1ull << cbits) - 1;
    const uint64_t fm = (fbits >= 64) ? ~0ull : ((1ull << fbits) - 1);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < F;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (!headflag[q]) continue;
        const uint64_t rc = keys[q] >> fbits;
        uint64_t r = vals[keys[q] & fm];
        for (int64_t x = q + 1; x < F && (keys[x] >> fbits) == rc; x++)
            r = sem_add(s, r, vals[keys[x] & fm]);
        const int64_t o = pos[q];
        ci[o] = (int32_t)(rc & cm);
        vout[o] = r;
        rows_key[o] = rc >> cbits;   // row id
    }
}

__global__ void k_rowptr_from_rows(const uint64_t *__restrict__ rows, int64_t nnz, int64_t nrows,
                                   int64_t *__restrict__ rp)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)rows[mid] < r) lo = mid + 1;
            else hi = mid;
        }
        rp[r] = lo;
    }
}

// ------------------------------------------------------------ eWise

template <bool UNION>
__global__ void k_ewise(const Csr A, const Csr B, int op, int vk, int akind, int bkind,
                        const int64_t *__restrict__ off, int64_t *__restrict__ cnt,
                        int32_t *__restrict__ ci, uint64_t *__restrict__ val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = A.rp[i], ae = A.rp[i + 1], b = B.rp[i], be = B.rp[i + 1];
        int64_t o = off ? off[i] : 0, c = 0;
        while (a < ae || b < be) {
            const int32_t ka = a < ae ? A.ci[a] : INT32_MAX;
            const int32_t kb = b < be ? B.ci[b] : INT32_MAX;
            int32_t j;
            uint64_t v = 0;
            bool emit;
            if (ka == kb) {
                j = ka;
                if (off)
                    v = binop(op, vk, convert(load_val(A.val, a, akind), akind, vk),
                              convert(load_val(B.val, b, bkind), bkind, vk));
                a++;
                b++;
                emit = true;
            } else if (ka < kb) {
                j = ka;
                if (off) v = convert(load_val(A.val, a, akind), akind, vk);
                a++;
                emit = UNION;
            } else {
                j = kb;
                if (off) v = convert(load_val(B.val, b, bkind), bkind, vk);
                b++;
                emit = UNION;
            }
            if (!emit) continue;
            if (off) {
                ci[o] = j;
                val[o] = v;
                o++;
            }
            c++;
        }
        if (!off) cnt[i] = c;
    }
}

// ------------------------------------------------------- reduce to vector

__global__ void k_row_reduce(const Csr A, int monoid, int vk, int akind, int64_t *__restrict__ has,
                             uint64_t *__restrict__ val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = A.rp[i], e = A.rp[i + 1];
        has[i] = e > a ? 1 : 0;
        if (e == a) continue;
        uint64_t r = convert(load_val(A.val, a, akind), akind, vk);
        for (int64_t p = a + 1; p < e; p++)
            r = binop(monoid, vk, r, convert(load_val(A.val, p, akind), akind, vk));
        val[i] = r;
    }
}

__global__ void k_vec_from_rows(const int64_t *__restrict__ has, const int64_t *__restrict__ pos,
                                const uint64_t *__restrict__ val, int64_t n, int32_t *__restrict__ ci,
                                uint64_t *__restrict__ vout)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!has[i]) continue;
        ci[pos[i]] = (int32_t)i;
        vout[pos[i]] = val[i];
    }
}

// ------------------------------------------------------ reduce to scalar

constexpr int RED_BLOCK = 256;
constexpr int RED_TILE = 4096;

// fixed order: each tile of RED_TILE consecutive entries is reduced by a
// fixed tree, then the tile partials left to right on the host side of the
// second pass
__global__ void k_tile_reduce(const uint64_t *__restrict__ vals, int64_t n, int monoid, int vk,
                              int from_kind, uint64_t *__restrict__ part)
{
    __shared__ uint64_t s[RED_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * RED_TILE;
    const int64_t end = base + RED_TILE < n ? base + RED_TILE : n;
    uint64_t r = 0;
    bool have = false;
    for (int64_t p = base + threadIdx.x; p < end; p += RED_BLOCK) {
        const uint64_t x = convert(load_val(vals, p, from_kind), from_kind, vk);
        r = have ? binop(monoid, vk, r, x) : x;
        have = true;
    }
    // identity fill for empty lanes: only lanes with values take part
    __shared__ int hv[RED_BLOCK];
    s[threadIdx.x] = r;
    hv[threadIdx.x] = have ? 1 : 0;
    __syncthreads();
    for (int w = RED_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (hv[o]) {
                s[threadIdx.x] = hv[threadIdx.x] ? binop(monoid, vk, s[threadIdx.x], s[o]) : s[o];
                hv[threadIdx.x] = 1;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_final_reduce(const uint64_t *__restrict__ part, int64_t n, int monoid, int vk,
                               uint64_t *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint64_t r = part[0];
        for (int64_t i = 1; i < n; i++) r = binop(monoid, vk, r, part[i]);
        *out = r;
    }
}

// ------------------------------------------------------------ write step

struct WriteArgs {
    Csr C, T, M;
    int has_mask, structural, comp, replace, accum, vk;
    int tkind;   // kind of T's values
};

// one merge of row i of C, T and the mask; count only when ci == nullptr
__device__ int64_t write_row(const WriteArgs &w, int64_t i, int32_t *ci, uint64_t *val, int64_t o)
{
    int64_t c = w.C.rp[i], ce = w.C.rp[i + 1], t = w.T.rp[i], te = w.T.rp[i + 1];
    int64_t m = w.has_mask ? w.M.rp[i] : 0, me = w.has_mask ? w.M.rp[i + 1] : 0;
    int64_t n = 0;
    while (c < ce || t < te) {
        const int32_t kc = c < ce ? w.C.ci[c] : INT32_MAX;
        const int32_t kt = t < te ? w.T.ci[t] : INT32_MAX;
        const int32_t j = kc < kt ? kc : kt;
        const bool inC = kc == j, inT = kt == j;
        // mask at j
        bool on = true;
        if (w.has_mask) {
            while (m < me && w.M.ci[m] < j) m++;
            on = m < me && w.M.ci[m] == j;
            if (on && !w.structural && w.M.val) on = mask_value_true(w.M, m);
        }
        if (w.comp) on = !on;
        uint64_t cv = inC ? load_val(w.C.val, c, w.vk) : 0;
        uint64_t tv = inT ? convert(load_val(w.T.val, t, w.tkind), w.tkind, w.vk) : 0;
        bool out = false;
        uint64_t ov = 0;
        if (on) {
            if (w.accum) {
                if (inC && inT) {
                    out = true;
                    ov = binop(w.accum, w.vk, cv, tv);
                } else if (inC) {
                    out = true;
                    ov = cv;
                } else if (inT) {
                    out = true;
                    ov = tv;
                }
            } else if (inT) {
                out = true;
                ov = tv;
            }
        } else if (!w.replace && inC) {
            out = true;
            ov = cv;
        }
        if (out) {
            if (ci) {
                ci[o + n] = j;
                if (val) val[o + n] = ov;
            }
            n++;
        }
        if (inC) c++;
        if (inT) t++;
    }
    return n;
}

__global__ void k_write_count(WriteArgs w, int64_t *__restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w.C.nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        cnt[i] = write_row(w, i, nullptr, nullptr, 0);
}

__global__ void k_write_fill(WriteArgs w, const int64_t *__restrict__ off, int32_t *__restrict__ ci,
                             uint64_t *__restrict__ val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w.C.nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        write_row(w, i, ci, val, off[i]);
}

// dense (bitmap) vector from a 1-row CSR
__global__ void k_scatter_dense(const Csr V, uint8_t *__restrict__ present, uint64_t *__restrict__ vals)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < V.nvals;
         q += (int64_t)gridDim.x * blockDim.x) {
        present[V.ci[q]] = 1;
        if (vals && V.val) vals[V.ci[q]] = V.val[q];
    }
}

// ------------------------------- plus.first under a complemented mask
//
// C<!s(M), r> = A plus.first B' with A of at most 64 rows (Algorithm 3's
// forward step F<!s(P), r> = F plus.first A, one source per row): the rows
// of A become the lanes of a wavefront.  A's entries are scattered into a
// dense k x 64 table with a lane mask per k, M's into a lane mask per
// output column; one wavefront per output column j then walks row j of
// B'^T (ascending k) and each lane adds the terms of its row -- the
// ascending-k order of the general path, so the same bits.  The result's
// lane masks are turned into C's rows by per-lane counts over 64-column
// tiles, one scan, and a write pass.

__device__ __forceinline__ uint64_t lane_shfl64(uint64_t x, int src)
{
    const unsigned lo = __shfl((unsigned)(x & 0xffffffffu), src, 64);
    const unsigned hi = __shfl((unsigned)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// blockIdx.y = row l: table[k][l] = value (when table), mask[k] |= 1 << l
__global__ void k_lane_scatter(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const uint64_t *__restrict__ val, int vk, uint64_t *__restrict__ table,
                               unsigned long long *__restrict__ mask)
{
    const int l = blockIdx.y;
    const int64_t b = rp[l], e = rp[l + 1];
    for (int64_t p = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < e; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = ci[p];
        if (table) table[k * 64 + l] = load_val(val, p, vk);
        atomicOr(mask + k, 1ull << l);
    }
}

__global__ __launch_bounds__(256) void k_lane_pull(const int64_t *__restrict__ brp, const int32_t *__restrict__ bci,
                                                   int64_t nj, uint64_t rows, const uint64_t *__restrict__ table,
                                                   const unsigned long long *__restrict__ fmask,
                                                   const unsigned long long *__restrict__ mmask, int fk, int ok,
                                                   unsigned long long *__restrict__ omask, uint64_t *__restrict__ oval)
{
    const unsigned lane = threadIdx.x & 63u;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < nj; j += nw) {
        const uint64_t adm = ~(uint64_t)mmask[j] & rows;
        uint64_t acc = ok == VK_F64 ? f_bits(0.0) : 0ull;
        bool have = false;
        if (adm) {
            const int64_t b = brp[j], e = brp[j + 1];
            for (int64_t p0 = b; p0 < e; p0 += 64) {
                const int64_t p = p0 + lane;
                int32_t k = 0;
                uint64_t hm = 0;
                if (p < e) {
                    k = bci[p];
                    hm = (uint64_t)fmask[k] & adm;
                }
                uint64_t hits = __ballot(hm != 0);
                while (hits) {
                    const int t = __ffsll((unsigned long long)hits) - 1;
                    hits &= hits - 1;
                    const int32_t kk = __shfl(k, t, 64);
                    const uint64_t mm = lane_shfl64(hm, t);
                    if ((mm >> lane) & 1ull) {
                        const uint64_t x = convert(table[(int64_t)kk * 64 + lane], fk, ok);
                        acc = have ? (ok == VK_F64 ? f_bits(bits_f(acc) + bits_f(x)) : acc + x) : x;
                        have = true;
                    }
                }
            }
        }
        const uint64_t hv = __ballot(have);
        if (lane == 0) omask[j] = hv;
        if (have) oval[j * 64 + lane] = ok == VK_I32 ? wrap32((int64_t)acc) : acc;
    }
}

// cnt[l * ntiles + t] = outputs of row l in columns [64 t, 64 t + 64)
__global__ __launch_bounds__(256) void k_lane_count(const unsigned long long *__restrict__ omask, int64_t nj,
                                                    int ns, int64_t *__restrict__ cnt)
{
    const unsigned lane = threadIdx.x & 63u;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (nj + 63) / 64;
    for (int64_t t = wave; t < ntiles; t += nw) {
        const int64_t j = t * 64 + lane;
        const uint64_t om = j < nj ? (uint64_t)omask[j] : 0ull;
        int mine = 0;
        for (int l = 0; l < ns; l++) {
            const int c = __popcll(__ballot((om >> l) & 1ull));
            if ((int)lane == l) mine = c;
        }
        if ((int)lane < ns) cnt[(int64_t)lane * ntiles + t] = mine;
    }
}

__global__ void k_lane_rowptr(const int64_t *__restrict__ pos, int64_t ntiles, int ns, int64_t total,
                              int64_t *__restrict__ rp)
{
    const int l = threadIdx.x;
    if (l < ns) rp[l] = ntiles > 0 ? pos[(int64_t)l * ntiles] : 0;
    if (l == ns) rp[ns] = total;
}

__global__ __launch_bounds__(256) void k_lane_write(const unsigned long long *__restrict__ omask,
                                                    const uint64_t *__restrict__ oval, int64_t nj, int ns,
                                                    const int64_t *__restrict__ pos, int32_t *__restrict__ ci,
                                                    uint64_t *__restrict__ val)
{
    const unsigned lane = threadIdx.x & 63u;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (nj + 63) / 64;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t t = wave; t < ntiles; t += nw) {
        const int64_t j = t * 64 + lane;
        const uint64_t om = j < nj ? (uint64_t)omask[j] : 0ull;
        for (int l = 0; l < ns; l++) {
            const bool on = (om >> l) & 1ull;
            const uint64_t b = __ballot(on);
            if (on) {
                const int64_t q = pos[(int64_t)l * ntiles + t] + __popcll(b & below);
                ci[q] = (int32_t)j;
                val[q] = oval[j * 64 + l];
            }
        }
    }
}

}  // namespace

// =============================================================== host side

namespace {

// Per-call device allocations.  When the owner goes out of scope they are
// handed to the context's deferred frees, so the call need not wait for
// the kernels that read them.
struct Pool {
    struct Blk {
        void *p;
        size_t n;
    };
    lagr_ctx ctx;
    Blk blks[48];
    int nb = 0;
    explicit Pool(lagr_ctx c) : ctx(c) {}
    void *get(size_t bytes)
    {
        if (bytes == 0) bytes = 8;
        if (nb >= 48) return nullptr;
        void *p = dev_alloc(bytes);
        if (p) blks[nb++] = {p, bytes};
        return p;
    }
    // hand ownership of p to the caller
    void release(void *p)
    {
        for (int i = 0; i < nb; i++)
            if (blks[i].p == p) {
                blks[i] = blks[--nb];
                return;
            }
    }
    ~Pool()
    {
        for (int i = 0; i < nb; i++) defer_free(ctx, blks[i].p, blks[i].n);
    }
};

int vkind_of(lagr_type t) { return t == LAGR_FP64 ? VK_F64 : t == LAGR_INT32 ? VK_I32 : VK_I64; }

Csr view(const lagr_matrix A)
{
    Csr c;
    c.nrows = A->nrows;
    c.ncols = A->ncols;
    c.nvals = A->nvals;
    c.rp = A->rowptr;
    c.ci = A->colidx;
    c.val = (const uint64_t *)A->values;
    c.type = A->type;
    return c;
}

#define G1(n) dim3(grid_for((n) > 0 ? (n) : 1, 256, 16384)), dim3(256), 0, ctx->stream

// 1 x n CSR of a vector (SPARSE: wrap; BITMAP / FULL: compacted copy)
int vec_view(lagr_ctx ctx, const lagr_vector v, Pool &pool, Csr *out, char *msg)
{
    Csr c;
    c.nrows = 1;
    c.ncols = v->n;
    c.type = v->type;
    int64_t *rp = (int64_t *)pool.get(16);
    if (!rp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector view");
    if (v->fmt == LAGR_VEC_SPARSE) {
        c.nvals = v->nvals;
        c.ci = v->idx;
        c.val = (const uint64_t *)v->values;
    } else {
        int64_t nv = 0;
        TRY(vector_tuples(ctx, v, nullptr, nullptr, &nv, msg));
        int32_t *ci = (int32_t *)pool.get(sizeof(int32_t) * (nv > 0 ? nv : 1));
        uint64_t *va = v->type != LAGR_BOOL ? (uint64_t *)pool.get(8 * (nv > 0 ? nv : 1)) : nullptr;
        if (!ci || (v->type != LAGR_BOOL && !va)) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector view");
        TRY(vector_tuples(ctx, v, ci, va, &nv, msg));
        c.nvals = nv;
        c.ci = ci;
        c.val = va;
    }
    hipLaunchKernelGGL(k_two, dim3(1), dim3(1), 0, ctx->stream, rp, (int64_t)0, c.nvals);
    LAUNCH_CHECK();
    c.rp = rp;
    *out = c;
    return LAGR_SUCCESS;
}

int transpose(lagr_ctx ctx, const Csr &A, Pool &pool, Csr *out, char *msg)
{
    Csr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.nvals = A.nvals;
    T.type = A.type;
    const int ebits = bits_for((uint64_t)(A.nvals > 0 ? A.nvals - 1 : 0));
    const int cbits = bits_for((uint64_t)(A.ncols > 0 ? A.ncols - 1 : 0));
    if (ebits + cbits > 64) return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "transpose too large");
    int64_t *rp = (int64_t *)pool.get(sizeof(int64_t) * (T.nrows + 1));
    int32_t *ci = (int32_t *)pool.get(sizeof(int32_t) * (A.nvals > 0 ? A.nvals : 1));
    uint64_t *va = A.val ? (uint64_t *)pool.get(8 * (A.nvals > 0 ? A.nvals : 1)) : nullptr;
    uint64_t *keys = (uint64_t *)pool.get(8 * (A.nvals > 0 ? A.nvals : 1));
    if (!rp || !ci || !keys || (A.val && !va)) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "transpose");
    if (A.nvals > 0) {
        hipLaunchKernelGGL(k_tr_keys, G1(A.nvals), A, ebits, keys);
        LAUNCH_CHECK();
        TRY(radix_sort_u64(ctx, keys, A.nvals, ebits + cbits, msg));
        hipLaunchKernelGGL(k_tr_fill, G1(A.nvals), A, keys, ebits, ci, va);
        LAUNCH_CHECK();
    }
    TRY(rowptr_from_sorted_keys(ctx, keys, A.nvals, ebits, T.nrows, rp, msg));
    T.rp = rp;
    T.ci = ci;
    T.val = va;
    *out = T;
    return LAGR_SUCCESS;
}

// compaction of dot-form results on M's pattern into a CSR T
int compact_on_mask(lagr_ctx ctx, const Csr &M, const uint8_t *has, const uint64_t *vals, Pool &pool,
                    lagr_type ttype, Csr *out, char *msg)
{
    int64_t *pos = (int64_t *)pool.get(sizeof(int64_t) * (M.nvals + 1));
    if (!pos) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "compaction");
    int64_t total = 0;
    if (M.nvals > 0) {
        hipLaunchKernelGGL(k_flags_i64, G1(M.nvals), has, M.nvals, pos);
        LAUNCH_CHECK();
    }
    TRY(scan_exclusive_i64(ctx, pos, pos, M.nvals, &total, msg));
    int32_t *ci = (int32_t *)pool.get(sizeof(int32_t) * (total > 0 ? total : 1));
    uint64_t *va = (uint64_t *)pool.get(8 * (total > 0 ? total : 1));
    int64_t *rp = (int64_t *)pool.get(sizeof(int64_t) * (M.nrows + 1));
    if (!ci || !va || !rp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "compaction");
    if (M.nvals > 0) {
        hipLaunchKernelGGL(k_compact, G1(M.nvals), M, has, pos, vals, ci, va);
        LAUNCH_CHECK();
    }
    // pos[M.nvals] = total serves the rows that start at the end
    TRY(fill_i64(ctx, pos + M.nvals, 1, total, msg));
    hipLaunchKernelGGL(k_rowptr_compacted, G1(M.nrows + 1), M, pos, total, rp);
    LAUNCH_CHECK();
    Csr T;
    T.nrows = M.nrows;
    T.ncols = M.ncols;
    T.nvals = total;
    T.rp = rp;
    T.ci = ci;
    T.val = va;
    T.type = ttype;
    *out = T;
    return LAGR_SUCCESS;
}

lagr_type sem_type(lagr_semiring s, lagr_type atype)
{
    switch (s) {
    case LAGR_PLUS_PAIR:
    case LAGR_ANY_SECONDI: return LAGR_INT64;
    case LAGR_PLUS_FIRST: return atype == LAGR_BOOL ? LAGR_INT64 : atype;
    default: return LAGR_FP64;
    }
}

// T = A' (+).(x) B' on the positions a (complemented) mask may keep
int product(lagr_ctx ctx, const Csr &A2, const Csr &B2, const Csr *B2T, const Csr *M, bool structural,
            bool comp, lagr_semiring semiring, Pool &pool, Csr *T, char *msg)
{
    const lagr_type ttype = sem_type(semiring, A2.type);
    Sem s;
    s.semiring = semiring;
    s.okind = vkind_of(ttype);
    s.astore = vkind_of(A2.type);
    s.bstore = vkind_of(B2.type);
    s.akind = semiring == LAGR_MIN_PLUS ? VK_F64 : s.astore;
    s.bkind = semiring == LAGR_MIN_PLUS ? VK_F64 : s.bstore;
    if (M && !comp) {
        // dot form: needs the rows of B'^T (given, or transposed here)
        Csr BT;
        if (B2T) BT = *B2T;
        else TRY(transpose(ctx, B2, pool, &BT, msg));
        uint64_t *vals = (uint64_t *)pool.get(8 * (M->nvals > 0 ? M->nvals : 1));
        uint8_t *has = (uint8_t *)pool.get(M->nvals > 0 ? M->nvals : 1);
        if (!vals || !has) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "dot form");
        const int valued = !structural && M->val != nullptr;
        if (semiring == LAGR_PLUS_PAIR && M->nvals > 0) {
            int64_t *cnt = (int64_t *)pool.get(8 * M->nvals);
            unsigned long long *tot = (unsigned long long *)pool.get(64);
            if (!cnt || !tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "dot form");
            TcArgs a;
            a.nrows = M->nrows;
            a.Mrp = M->rp;
            a.Mci = M->ci;
            a.Arp = A2.rp;
            a.Aci = A2.ci;
            a.Brp = BT.rp;
            a.Bci = BT.ci;
            a.tc_form = 0;
            TRY(tc_masked_dot(ctx, a, true, tot, cnt, msg));
            hipLaunchKernelGGL(k_counts_to_has, G1(M->nvals), cnt, M->nvals, *M, valued, vals, has);
            LAUNCH_CHECK();
        } else if (M->nvals > 0) {
            Sem sd = s;
            hipLaunchKernelGGL(k_dot, G1(M->nvals), *M, A2, BT, valued, sd, vals, has);
            LAUNCH_CHECK();
        }
        return compact_on_mask(ctx, *M, has, vals, pool, ttype, T, msg);
    }
    // saxpy form
    int64_t *fl = (int64_t *)pool.get(sizeof(int64_t) * (A2.nrows + 1));
    if (!fl) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "saxpy");
    TRY(fill_i64(ctx, fl + A2.nrows, 1, 0, msg));
    if (A2.nrows > 0) {
        hipLaunchKernelGGL(k_flops, G1(A2.nrows), A2, B2, fl);
        LAUNCH_CHECK();
    }
    int64_t F = 0;
    TRY(scan_exclusive_i64(ctx, fl, fl, A2.nrows + 1, &F, msg));
    const int rbits = bits_for((uint64_t)(A2.nrows > 0 ? A2.nrows - 1 : 0));
    const int cbits = bits_for((uint64_t)(B2.ncols > 0 ? B2.ncols - 1 : 0)) + 0;
    const int cb = cbits > 0 ? cbits : 1;
    const int fbits = bits_for((uint64_t)(F > 0 ? F - 1 : 0)) > 0 ? bits_for((uint64_t)(F - 1)) : 1;
    if (rbits + cb + fbits > 64)
        return lagr_fail(msg, LAGR_NOT_IMPLEMENTED, "product too large for the saxpy form (%lld terms)",
                         (long long)F);
    uint64_t *keys = (uint64_t *)pool.get(8 * (F > 0 ? F : 1));
    uint64_t *vals = (uint64_t *)pool.get(8 * (F > 0 ? F : 1));
    int64_t *head = (int64_t *)pool.get(8 * (F + 1));
    if (!keys || !vals || !head) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "saxpy products");
    if (A2.nrows > 0 && F > 0) {
        hipLaunchKernelGGL(k_expand, G1(A2.nrows), A2, B2, fl, s, cb, fbits, keys, vals);
        LAUNCH_CHECK();
    }
    TRY(radix_sort_u64(ctx, keys, F, rbits + cb + fbits, msg));
    Csr Mv;
    if (M) Mv = *M;
    if (F > 0) {
        hipLaunchKernelGGL(k_run_heads, G1(F), keys, F, fbits, cb, Mv, M ? 1 : 0, structural ? 1 : 0,
                           comp ? 1 : 0, head);
        LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    TRY(scan_exclusive_i64(ctx, head, head, F, &nnz, msg));
    // the flags were overwritten by their prefix; recompute them
    int64_t *flag = (int64_t *)pool.get(8 * (F + 1));
    int32_t *ci = (int32_t *)pool.get(4 * (nnz > 0 ? nnz : 1));
    uint64_t *va = (uint64_t *)pool.get(8 * (nnz > 0 ? nnz : 1));
    uint64_t *rows = (uint64_t *)pool.get(8 * (nnz > 0 ? nnz : 1));
    int64_t *rp = (int64_t *)pool.get(8 * (A2.nrows + 1));
    if (!flag || !ci || !va || !rows || !rp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "saxpy output");
    if (F > 0) {
        hipLaunchKernelGGL(k_run_heads, G1(F), keys, F, fbits, cb, Mv, M ? 1 : 0, structural ? 1 : 0,
                           comp ? 1 : 0, flag);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_runs_reduce, G1(F), keys, vals, F, fbits, cb, head, flag, s, ci, va, rows);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_rowptr_from_rows, G1(A2.nrows + 1), rows, nnz, A2.nrows, rp);
    LAUNCH_CHECK();
    Csr R;
    R.nrows = A2.nrows;
    R.ncols = B2.ncols;
    R.nvals = nnz;
    R.rp = rp;
    R.ci = ci;
    R.val = va;
    R.type = ttype;
    *T = R;
    return LAGR_SUCCESS;
}

// C<M> accum= T (all rules); result arrays returned through *out (owned by
// the caller from then on)
struct NewCsr {
    int64_t *rp;
    int32_t *ci;
    uint64_t *val;
    int64_t nnz;
    size_t rb, cb, vb;
};

int write_step(lagr_ctx ctx, const Csr &C, const Csr &T, const Csr *M, uint32_t desc, lagr_binop accum,
               Pool &pool, NewCsr *out, char *msg)
{
    WriteArgs w;
    w.C = C;
    w.T = T;
    if (M) w.M = *M;
    w.has_mask = M ? 1 : 0;
    w.structural = (desc & LAGR_DESC_STRUCT) ? 1 : 0;
    w.comp = (desc & LAGR_DESC_COMP) ? 1 : 0;
    w.replace = (desc & LAGR_DESC_REPLACE) ? 1 : 0;
    w.accum = accum;
    w.vk = vkind_of(C.type);
    w.tkind = vkind_of(T.type);
    int64_t *off = (int64_t *)pool.get(8 * (C.nrows + 1));
    if (!off) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "write step");
    TRY(fill_i64(ctx, off + C.nrows, 1, 0, msg));
    if (C.nrows > 0) {
        hipLaunchKernelGGL(k_write_count, G1(C.nrows), w, off);
        LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    TRY(scan_exclusive_i64(ctx, off, off, C.nrows + 1, &nnz, msg));
    NewCsr r;
    r.nnz = nnz;
    r.rb = 8 * (C.nrows + 1);
    r.cb = 4 * (nnz > 0 ? nnz : 1);
    r.vb = C.type == LAGR_BOOL ? 0 : 8 * (nnz > 0 ? nnz : 1);
    r.rp = (int64_t *)dev_alloc(r.rb);
    r.ci = (int32_t *)dev_alloc(r.cb);
    r.val = r.vb ? (uint64_t *)dev_alloc(r.vb) : nullptr;
    if (!r.rp || !r.ci || (r.vb && !r.val)) {
        dev_free(r.rp, r.rb);
        dev_free(r.ci, r.cb);
        dev_free(r.val, r.vb);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "result arrays");
    }
    HIP_TRY(hipMemcpyAsync(r.rp, off, r.rb, hipMemcpyDeviceToDevice, ctx->stream));
    if (C.nrows > 0) {
        hipLaunchKernelGGL(k_write_fill, G1(C.nrows), w, off, r.ci, r.val);
        LAUNCH_CHECK();
    }
    *out = r;
    return LAGR_SUCCESS;
}

void install_matrix(lagr_ctx ctx, lagr_matrix C, const NewCsr &r)
{
    // queued kernels may still read C's old arrays (C may be an input)
    matrix_release_arrays_later(ctx, C);
    C->rowptr = r.rp;
    C->colidx = r.ci;
    C->values = r.val;
    C->rowptr_bytes = r.rb;
    C->colidx_bytes = r.cb;
    C->values_bytes = r.vb;
    C->nvals = r.nnz;
}

// store a 1-row result into vector w, keeping its storage class
int install_vector(lagr_ctx ctx, lagr_vector w, const NewCsr &r, char *msg)
{
    // queued kernels may still read w's old arrays (w may be an input)
    if (w->fmt == LAGR_VEC_SPARSE) {
        vector_release_arrays_later(ctx, w);
        w->idx = r.ci;
        w->idx_bytes = r.cb;
        w->values = r.val;
        w->values_bytes = r.vb;
        w->nvals = r.nnz;
        defer_free(ctx, r.rp, r.rb);
        return LAGR_SUCCESS;
    }
    const int64_t n = w->n;
    uint8_t *pres = (uint8_t *)dev_alloc(n > 0 ? n : 1);
    uint64_t *vals = w->type != LAGR_BOOL ? (uint64_t *)dev_alloc(8 * (n > 0 ? n : 1)) : nullptr;
    if (!pres || (w->type != LAGR_BOOL && !vals)) {
        dev_free(pres, n > 0 ? n : 1);
        dev_free(vals, 8 * (n > 0 ? n : 1));
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "vector arrays");
    }
    TRY(fill_u8(ctx, pres, n, 0, msg));
    Csr V;
    V.nrows = 1;
    V.ncols = n;
    V.nvals = r.nnz;
    V.rp = r.rp;
    V.ci = r.ci;
    V.val = r.val;
    if (r.nnz > 0) {
        hipLaunchKernelGGL(k_scatter_dense, G1(r.nnz), V, pres, vals);
        LAUNCH_CHECK();
    }
    defer_free(ctx, r.rp, r.rb);
    defer_free(ctx, r.ci, r.cb);
    defer_free(ctx, r.val, r.vb);
    vector_release_arrays_later(ctx, w);
    w->values = vals;
    w->values_bytes = vals ? 8 * (size_t)(n > 0 ? n : 1) : 0;
    if (w->fmt == LAGR_VEC_FULL && r.nnz == n && w->type != LAGR_BOOL) {
        dev_free(pres, n > 0 ? n : 1);
        w->nvals = n;
    } else {
        w->fmt = LAGR_VEC_BITMAP;
        w->present = pres;
        w->present_bytes = (size_t)(n > 0 ? n : 1);
        w->nvals = -1;
    }
    return LAGR_SUCCESS;
}

int check_desc(uint32_t desc, char *msg)
{
    const uint32_t known = LAGR_DESC_COMP | LAGR_DESC_STRUCT | LAGR_DESC_REPLACE | LAGR_DESC_TRAN0 |
                           LAGR_DESC_TRAN1 | LAGR_DESC_DETERMINISTIC | LAGR_DESC_ASSIGN_PARENT;
    if (desc & ~known) return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown descriptor bits 0x%x", desc);
    return LAGR_SUCCESS;
}

int check_accum(lagr_binop accum, lagr_type ctype, char *msg)
{
    if ((int)accum < 0 || (int)accum > (int)LAGR_ANY)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown accumulator %d", (int)accum);
    if (accum != LAGR_NOOP && ctype == LAGR_BOOL)
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "an accumulator needs a valued output");
    if (accum == LAGR_DIV && ctype != LAGR_FP64)
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "DIV is defined on FP64 only");
    return LAGR_SUCCESS;
}

int check_semiring(lagr_semiring s, char *msg)
{
    if ((int)s < 0 || (int)s > (int)LAGR_MIN_PLUS)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown semiring %d", (int)s);
    return LAGR_SUCCESS;
}

}  // namespace

int matrix_transpose(lagr_ctx ctx, const lagr_matrix A, lagr_matrix *out, char *msg)
{
    *out = nullptr;
    Pool pool(ctx);
    Csr T;
    TRY(transpose(ctx, view(A), pool, &T, msg));
    lagr_matrix M = new (std::nothrow) lagr_matrix_s();
    if (!M) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "matrix");
    M->type = A->type;
    M->nrows = A->ncols;
    M->ncols = A->nrows;
    M->nvals = A->nvals;
    M->rowptr = (int64_t *)T.rp;
    M->colidx = (int32_t *)T.ci;
    M->values = (void *)T.val;
    M->rowptr_bytes = sizeof(int64_t) * (size_t)(M->nrows + 1);
    M->colidx_bytes = sizeof(int32_t) * (size_t)(M->nvals > 0 ? M->nvals : 1);
    M->values_bytes = T.val ? 8 * (size_t)(M->nvals > 0 ? M->nvals : 1) : 0;
    pool.release((void *)T.rp);
    pool.release((void *)T.ci);
    if (T.val) pool.release((void *)T.val);
    // (the pool's sort keys are freed once the queued kernels are done)
    *out = M;
    return LAGR_SUCCESS;
}

// Rows of A^T: A's cached transpose, built by the first call that needs it.
// A matrix is not written while a call reads it, so the cache stays valid
// until its arrays are replaced; the lock covers two threads asking for
// the same matrix's transpose at once.
int cached_transpose(lagr_ctx ctx, const lagr_matrix A, Csr *out, char *msg)
{
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (!A->tcache) TRY(matrix_transpose(ctx, A, &A->tcache, msg));
    *out = view(A->tcache);
    return LAGR_SUCCESS;
}

// C<!s(M), r> = A plus.first B' on lanes (A has at most 64 rows, no
// accumulator; C is replaced, or empty).  Returns 1 when computed, 0 when
// the call has another shape, < 0 on error.
static int mxm_plus_first_lanes(lagr_ctx ctx, lagr_matrix C, const lagr_matrix M, lagr_binop accum,
                                lagr_semiring semiring, const lagr_matrix A, const lagr_matrix B, uint32_t desc,
                                char *msg)
{
    const uint32_t sc = LAGR_DESC_STRUCT | LAGR_DESC_COMP;
    if (semiring != LAGR_PLUS_FIRST || !M || (desc & sc) != sc || (desc & LAGR_DESC_TRAN0) || accum != LAGR_NOOP)
        return 0;
    if (A->nrows > 64 || A->nrows < 1 || ctx->device < 0) return 0;
    if (!(desc & LAGR_DESC_REPLACE) && C->nvals != 0) return 0;
    const int ns = (int)A->nrows;
    const int64_t nk = A->ncols, nj = C->ncols;
    const bool t1 = desc & LAGR_DESC_TRAN1;
    // rows of B'^T: B itself under TRAN1, else B's cached transpose
    Csr BT;
    if (t1) BT = view(B);
    else TRY(cached_transpose(ctx, B, &BT, msg));
    Pool pool(ctx);
    const size_t k1 = (size_t)(nk > 0 ? nk : 1), j1 = (size_t)(nj > 0 ? nj : 1);
    uint64_t *table = (uint64_t *)pool.get(8 * 64 * k1);
    unsigned long long *fmask = (unsigned long long *)pool.get(8 * k1);
    unsigned long long *mmask = (unsigned long long *)pool.get(8 * j1);
    unsigned long long *omask = (unsigned long long *)pool.get(8 * j1);
    uint64_t *oval = (uint64_t *)pool.get(8 * 64 * j1);
    const int64_t ntiles = (nj + 63) / 64;
    int64_t *pos = (int64_t *)pool.get(8 * ((size_t)ns * (size_t)ntiles + 1));
    if (!table || !fmask || !mmask || !omask || !oval || !pos) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "lanes");
    TRY(fill_i64(ctx, (int64_t *)fmask, nk, 0, msg));
    TRY(fill_i64(ctx, (int64_t *)mmask, nj, 0, msg));
    const int fk = vkind_of(A->type), ok = vkind_of(C->type);
    const unsigned sx = grid_for(nk > nj ? nk : nj, 256, 1024);
    if (A->nvals > 0) {
        hipLaunchKernelGGL(k_lane_scatter, dim3(sx, (unsigned)ns), dim3(256), 0, ctx->stream, A->rowptr, A->colidx,
                           (const uint64_t *)A->values, fk, table, fmask);
        LAUNCH_CHECK();
    }
    if (M->nvals > 0) {
        hipLaunchKernelGGL(k_lane_scatter, dim3(sx, (unsigned)ns), dim3(256), 0, ctx->stream, M->rowptr, M->colidx,
                           (const uint64_t *)nullptr, fk, (uint64_t *)nullptr, mmask);
        LAUNCH_CHECK();
    }
    const uint64_t rows = ns == 64 ? ~0ull : ((1ull << ns) - 1);
    if (nj > 0) {
        hipLaunchKernelGGL(k_lane_pull, dim3(grid_for(nj * 64, 256, 16384)), dim3(256), 0, ctx->stream, BT.rp, BT.ci,
                           nj, rows, table, fmask, mmask, fk, ok, omask, oval);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_lane_count, dim3(grid_for(ntiles * 64, 256, 16384)), dim3(256), 0, ctx->stream, omask,
                           nj, ns, pos);
        LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    TRY(scan_exclusive_i64(ctx, pos, pos, (int64_t)ns * ntiles, &nnz, msg));
    NewCsr r;
    r.nnz = nnz;
    r.rb = 8 * (size_t)(ns + 1);
    r.cb = 4 * (size_t)(nnz > 0 ? nnz : 1);
    r.vb = 8 * (size_t)(nnz > 0 ? nnz : 1);
    r.rp = (int64_t *)dev_alloc(r.rb);
    r.ci = (int32_t *)dev_alloc(r.cb);
    r.val = (uint64_t *)dev_alloc(r.vb);
    if (!r.rp || !r.ci || !r.val) {
        dev_free(r.rp, r.rb);
        dev_free(r.ci, r.cb);
        dev_free(r.val, r.vb);
        return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "result arrays");
    }
    hipLaunchKernelGGL(k_lane_rowptr, dim3(1), dim3(128), 0, ctx->stream, pos, ntiles, ns, nnz, r.rp);
    LAUNCH_CHECK();
    if (nnz > 0) {
        hipLaunchKernelGGL(k_lane_write, dim3(grid_for(ntiles * 64, 256, 16384)), dim3(256), 0, ctx->stream, omask,
                           oval, nj, ns, pos, r.ci, r.val);
        LAUNCH_CHECK();
    }
    install_matrix(ctx, C, r);
    return 1;
}

// =================================================================== API

extern "C" int lagr_mxm(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_semiring semiring,
                        const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!C || !A || !B || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    TRY(check_semiring(semiring, msg));
    const bool t0 = desc & LAGR_DESC_TRAN0, t1 = desc & LAGR_DESC_TRAN1;
    const int64_t am = t0 ? A->ncols : A->nrows, ak = t0 ? A->nrows : A->ncols;
    const int64_t bk = t1 ? B->ncols : B->nrows, bn = t1 ? B->nrows : B->ncols;
    if (ak != bk || C->nrows != am || C->ncols != bn)
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "A' is %lld x %lld, B' is %lld x %lld, C is %lld x %lld",
                         (long long)am, (long long)ak, (long long)bk, (long long)bn, (long long)C->nrows,
                         (long long)C->ncols);
    if (M && (M->nrows != C->nrows || M->ncols != C->ncols))
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask dimensions differ from C");
    const lagr_type tt = sem_type(semiring, A->type);
    if (C->type != tt)
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "C's type %d differs from the semiring result type %d",
                         (int)C->type, (int)tt);
    TRY(check_accum(accum, C->type, msg));
    {
        // Algorithm 3's forward step on its own kernels
        const int fast = mxm_plus_first_lanes(ctx, C, M, accum, semiring, A, B, desc, msg);
        if (fast < 0) return fast;
        if (fast) return lagr_ok(msg);
    }
    Pool pool(ctx);
    Csr A2 = view(A), B2 = view(B), B2T;
    // the dot form (a mask, not complemented) reads rows of B'^T, which is
    // B itself under TRAN1; the saxpy form reads rows of B'
    const bool dot = M && !(desc & LAGR_DESC_COMP);
    if (t0) TRY(cached_transpose(ctx, A, &A2, msg));
    if (dot) {
        if (t1) B2T = view(B);
        else TRY(cached_transpose(ctx, B, &B2T, msg));
    } else if (t1) {
        TRY(cached_transpose(ctx, B, &B2, msg));
    }
    Csr Mv;
    if (M) Mv = view(M);
    Csr T;
    TRY(product(ctx, A2, B2, dot ? &B2T : nullptr, M ? &Mv : nullptr, desc & LAGR_DESC_STRUCT,
                desc & LAGR_DESC_COMP, semiring, pool, &T, msg));
    NewCsr r;
    TRY(write_step(ctx, view(C), T, M ? &Mv : nullptr, desc, accum, pool, &r, msg));
    install_matrix(ctx, C, r);
    return lagr_ok(msg);
}

extern "C" int lagr_vxm(lagr_vector w, const lagr_vector m, lagr_binop accum, lagr_semiring semiring,
                        const lagr_vector u, const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!w || !u || !A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    TRY(check_semiring(semiring, msg));
    if (desc & LAGR_DESC_TRAN0) return lagr_fail(msg, LAGR_INVALID_VALUE, "vxm takes no TRAN0");
    const bool t1 = desc & LAGR_DESC_TRAN1;
    const int64_t ak = t1 ? A->ncols : A->nrows, an = t1 ? A->nrows : A->ncols;
    if (u->n != ak || w->n != an)
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "u has %lld entries, A' is %lld x %lld, w has %lld",
                         (long long)u->n, (long long)ak, (long long)an, (long long)w->n);
    if (m && m->n != w->n) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask length differs from w");
    const lagr_type tt = sem_type(semiring, u->type);
    if (w->type != tt) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "w's type differs from the result type");
    TRY(check_accum(accum, w->type, msg));
    if (desc & LAGR_DESC_ASSIGN_PARENT) {
        // the mask is the parent vector p, and receives p<s(w)> = w
        if (!m) return lagr_fail(msg, LAGR_NULL_POINTER, "ASSIGN_PARENT needs the parent vector as the mask");
        if (m->type != LAGR_INT64) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "the parent vector must be INT64");
    }
    {
        const int fast = vxm_any_secondi_fast(w, m, accum, semiring, u, A, desc, ctx, msg);
        if (fast < 0) return fast;
        if (fast) return lagr_ok(msg);
    }
    {
        Pool pool(ctx);
        Csr U, W, Mv, A2 = view(A), A2T;
        TRY(vec_view(ctx, u, pool, &U, msg));
        TRY(vec_view(ctx, w, pool, &W, msg));
        if (m) TRY(vec_view(ctx, m, pool, &Mv, msg));
        // as in lagr_mxm: the dot form reads rows of A'^T (A itself under
        // TRAN1), the saxpy form rows of A'
        const bool dot = m && !(desc & LAGR_DESC_COMP);
        if (dot) {
            if (t1) A2T = view(A);
            else TRY(cached_transpose(ctx, A, &A2T, msg));
        } else if (t1) {
            TRY(cached_transpose(ctx, A, &A2, msg));
        }
        Csr T;
        TRY(product(ctx, U, A2, dot ? &A2T : nullptr, m ? &Mv : nullptr, desc & LAGR_DESC_STRUCT,
                    desc & LAGR_DESC_COMP, semiring, pool, &T, msg));
        NewCsr r;
        TRY(write_step(ctx, W, T, m ? &Mv : nullptr, desc, accum, pool, &r, msg));
        TRY(install_vector(ctx, w, r, msg));
    }
    if (desc & LAGR_DESC_ASSIGN_PARENT) TRY(lagr_assign_vector(m, w, LAGR_NOOP, w, LAGR_DESC_STRUCT, ctx, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_mxm_reduce(void *s, const lagr_matrix M, lagr_semiring semiring, const lagr_matrix A,
                               const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!s || !A || !B || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    TRY(check_semiring(semiring, msg));
    const bool t0 = desc & LAGR_DESC_TRAN0, t1 = desc & LAGR_DESC_TRAN1;
    const int64_t am = t0 ? A->ncols : A->nrows, ak = t0 ? A->nrows : A->ncols;
    const int64_t bk = t1 ? B->ncols : B->nrows, bn = t1 ? B->nrows : B->ncols;
    if (ak != bk) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "inner dimensions differ");
    if (M && (M->nrows != am || M->ncols != bn))
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask dimensions differ from the product");
    const lagr_type tt = sem_type(semiring, A->type);
    const bool structural = (desc & LAGR_DESC_STRUCT) || (M && M->type == LAGR_BOOL);
    // fused: plus.pair dot form under a structural mask, on A and B as given
    if (semiring == LAGR_PLUS_PAIR && M && !(desc & LAGR_DESC_COMP) && structural && !t0 && t1) {
        unsigned long long *tot = (unsigned long long *)ws_get(ctx, WS_TC, 64);
        if (!tot) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "counter");
        TcArgs a;
        a.nrows = M->nrows;
        a.Mrp = M->rowptr;
        a.Mci = M->colidx;
        a.Arp = A->rowptr;
        a.Aci = A->colidx;
        a.Brp = B->rowptr;
        a.Bci = B->colidx;
        a.tc_form = 0;
        TRY(tc_masked_dot(ctx, a, false, tot, nullptr, msg));
        unsigned long long h = 0;
        TRY(read_back(ctx, &h, tot, 8, msg));
        *(int64_t *)s = (int64_t)h;
        return lagr_ok(msg);
    }
    // otherwise: form C, then reduce it with plus
    lagr_matrix C = nullptr;
    TRY(lagr_matrix_new(&C, tt, am, bn, ctx, msg));
    int rc = lagr_mxm(C, M, LAGR_NOOP, semiring, A, B, desc & ~LAGR_DESC_REPLACE, ctx, msg);
    if (rc >= 0) {
        if (tt == LAGR_FP64) *(double *)s = 0.0;
        else *(int64_t *)s = 0;
        rc = lagr_reduce_scalar(s, LAGR_NOOP, LAGR_PLUS, C, ctx, msg);
        if (rc == LAGR_NO_VALUE) rc = lagr_ok(msg);
    }
    lagr_matrix_free(&C);
    return rc;
}

static int reduce_values(lagr_ctx ctx, const uint64_t *vals, int64_t nv, lagr_type from, lagr_type to,
                         lagr_binop monoid, uint64_t *out, char *msg)
{
    Pool pool(ctx);
    const int64_t tiles = (nv + RED_TILE - 1) / RED_TILE;
    uint64_t *part = (uint64_t *)pool.get(8 * (tiles + 1));
    if (!part) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "reduce");
    hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)tiles), dim3(RED_BLOCK), 0, ctx->stream, vals, nv,
                       (int)monoid, vkind_of(to), vkind_of(from), part);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(64), 0, ctx->stream, part, tiles, (int)monoid,
                       vkind_of(to), part + tiles);
    LAUNCH_CHECK();
    return read_back(ctx, out, part + tiles, 8, msg);
}

static int scalar_result(void *s, lagr_binop accum, lagr_type t, uint64_t r)
{
    if (t == LAGR_FP64) {
        const double y = bits_f(r);
        double *x = (double *)s;
        switch (accum) {
        case LAGR_NOOP:
        case LAGR_SECOND: *x = y; break;
        case LAGR_PLUS: *x = *x + y; break;
        case LAGR_MIN: *x = y < *x ? y : *x; break;
        case LAGR_TIMES: *x = *x * y; break;
        case LAGR_DIV: *x = *x / y; break;
        default: break;   // FIRST / ANY keep s
        }
    } else if (t == LAGR_INT32) {
        // modulo 2^32, through unsigned arithmetic
        const uint32_t y = (uint32_t)r;
        int32_t *x = (int32_t *)s;
        switch (accum) {
        case LAGR_NOOP:
        case LAGR_SECOND: *x = (int32_t)y; break;
        case LAGR_PLUS: *x = (int32_t)((uint32_t)*x + y); break;
        case LAGR_MIN: *x = (int32_t)y < *x ? (int32_t)y : *x; break;
        case LAGR_TIMES: *x = (int32_t)((uint32_t)*x * y); break;
        default: break;
        }
    } else {
        const int64_t y = (int64_t)r;
        int64_t *x = (int64_t *)s;
        switch (accum) {
        case LAGR_NOOP:
        case LAGR_SECOND: *x = y; break;
        case LAGR_PLUS: *x = (int64_t)((uint64_t)*x + (uint64_t)y); break;
        case LAGR_MIN: *x = y < *x ? y : *x; break;
        case LAGR_TIMES: *x = (int64_t)((uint64_t)*x * (uint64_t)y); break;
        default: break;
        }
    }
    return LAGR_SUCCESS;
}

extern "C" int lagr_reduce_scalar(void *s, lagr_binop accum, lagr_binop monoid, const lagr_matrix A,
                                  lagr_ctx ctx, char *msg)
{
    if (!s || !A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (monoid != LAGR_PLUS && monoid != LAGR_MIN)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "the reduce monoid is PLUS or MIN");
    const lagr_type t = A->type == LAGR_BOOL ? LAGR_INT64 : A->type;
    TRY(check_accum(accum, t, msg));
    if (A->nvals == 0) {
        if (msg) snprintf(msg, LAGR_MSG_LEN, "no entries");
        return LAGR_NO_VALUE;
    }
    uint64_t r = 0;
    TRY(reduce_values(ctx, (const uint64_t *)A->values, A->nvals, A->type, t, monoid, &r, msg));
    scalar_result(s, accum, t, r);
    return lagr_ok(msg);
}

extern "C" int lagr_vector_reduce_scalar(void *s, lagr_binop accum, lagr_binop monoid, const lagr_vector u,
                                         lagr_ctx ctx, char *msg)
{
    if (!s || !u || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    if (monoid != LAGR_PLUS && monoid != LAGR_MIN)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "the reduce monoid is PLUS or MIN");
    const lagr_type t = u->type == LAGR_BOOL ? LAGR_INT64 : u->type;
    TRY(check_accum(accum, t, msg));
    Pool pool(ctx);
    Csr U;
    TRY(vec_view(ctx, u, pool, &U, msg));
    if (U.nvals == 0) {
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if (msg) snprintf(msg, LAGR_MSG_LEN, "no entries");
        return LAGR_NO_VALUE;
    }
    uint64_t r = 0;
    TRY(reduce_values(ctx, U.val, U.nvals, u->type, t, monoid, &r, msg));
    scalar_result(s, accum, t, r);
    return lagr_ok(msg);
}

extern "C" int lagr_reduce_rows(lagr_vector w, const lagr_vector m, lagr_binop accum, lagr_binop monoid,
                                const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!w || !A || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    if (monoid != LAGR_PLUS && monoid != LAGR_MIN)
        return lagr_fail(msg, LAGR_INVALID_VALUE, "the reduce monoid is PLUS or MIN");
    const bool t0 = desc & LAGR_DESC_TRAN0;
    const int64_t rows = t0 ? A->ncols : A->nrows;
    if (w->n != rows) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "w length differs from A' rows");
    if (m && m->n != w->n) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask length differs from w");
    const lagr_type t = A->type == LAGR_BOOL ? LAGR_INT64 : A->type;
    if (w->type != t) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "w's type differs from A's value type");
    TRY(check_accum(accum, w->type, msg));
    Pool pool(ctx);
    Csr A2 = view(A);
    if (t0) TRY(cached_transpose(ctx, A, &A2, msg));
    int64_t *has = (int64_t *)pool.get(8 * (rows + 1));
    uint64_t *val = (uint64_t *)pool.get(8 * (rows > 0 ? rows : 1));
    int64_t *rp = (int64_t *)pool.get(16);
    if (!has || !val || !rp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "reduce rows");
    if (rows > 0) {
        hipLaunchKernelGGL(k_row_reduce, G1(rows), A2, (int)monoid, vkind_of(t), vkind_of(A->type), has,
                           val);
        LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    int64_t *pos = (int64_t *)pool.get(8 * (rows + 1));
    if (!pos) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "reduce rows");
    HIP_TRY(hipMemcpyAsync(pos, has, 8 * (rows > 0 ? rows : 1), hipMemcpyDeviceToDevice, ctx->stream));
    TRY(scan_exclusive_i64(ctx, pos, pos, rows, &nnz, msg));
    int32_t *ci = (int32_t *)pool.get(4 * (nnz > 0 ? nnz : 1));
    uint64_t *vo = (uint64_t *)pool.get(8 * (nnz > 0 ? nnz : 1));
    if (!ci || !vo) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "reduce rows");
    if (rows > 0) {
        hipLaunchKernelGGL(k_vec_from_rows, G1(rows), has, pos, val, rows, ci, vo);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_two, dim3(1), dim3(1), 0, ctx->stream, rp, (int64_t)0, nnz);
    LAUNCH_CHECK();
    Csr T;
    T.nrows = 1;
    T.ncols = rows;
    T.nvals = nnz;
    T.rp = rp;
    T.ci = ci;
    T.val = vo;
    T.type = t;
    Csr W, Mv;
    TRY(vec_view(ctx, w, pool, &W, msg));
    if (m) TRY(vec_view(ctx, m, pool, &Mv, msg));
    NewCsr r;
    TRY(write_step(ctx, W, T, m ? &Mv : nullptr, desc, accum, pool, &r, msg));
    TRY(install_vector(ctx, w, r, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_assign_vector(lagr_vector w, const lagr_vector m, lagr_binop accum, const lagr_vector u,
                                  uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!w || !u || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    if (u->n != w->n) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "u and w lengths differ");
    if (m && m->n != w->n) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask length differs from w");
    if (w->type == LAGR_BOOL && u->type != LAGR_BOOL)
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "a BOOL vector cannot take values");
    TRY(check_accum(accum, w->type, msg));
    Pool pool(ctx);
    Csr U, W, Mv;
    TRY(vec_view(ctx, u, pool, &U, msg));
    TRY(vec_view(ctx, w, pool, &W, msg));
    if (m) TRY(vec_view(ctx, m, pool, &Mv, msg));
    NewCsr r;
    TRY(write_step(ctx, W, U, m ? &Mv : nullptr, desc, accum, pool, &r, msg));
    TRY(install_vector(ctx, w, r, msg));
    return lagr_ok(msg);
}

extern "C" int lagr_assign_scalar(lagr_vector w, const lagr_vector m, lagr_binop accum, const void *s,
                                  uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!w || !s || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    if (m && m->n != w->n) return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask length differs from w");
    if (w->type == LAGR_BOOL) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "a BOOL vector cannot take values");
    TRY(check_accum(accum, w->type, msg));
    Pool pool(ctx);
    const int64_t n = w->n;
    int32_t *ci = (int32_t *)pool.get(4 * (n > 0 ? n : 1));
    uint64_t *va = (uint64_t *)pool.get(8 * (n > 0 ? n : 1));
    int64_t *rp = (int64_t *)pool.get(16);
    if (!ci || !va || !rp) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "assign");
    uint64_t sv;
    if (w->type == LAGR_INT32) {
        int32_t s32;
        memcpy(&s32, s, 4);
        sv = (uint64_t)(int64_t)s32;
    } else {
        memcpy(&sv, s, 8);
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_iota32, G1(n), ci, n);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_fill_u64, G1(n), va, n, sv);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_two, dim3(1), dim3(1), 0, ctx->stream, rp, (int64_t)0, n);
    LAUNCH_CHECK();
    Csr T;
    T.nrows = 1;
    T.ncols = n;
    T.nvals = n;
    T.rp = rp;
    T.ci = ci;
    T.val = va;
    T.type = w->type;
    Csr W, Mv;
    TRY(vec_view(ctx, w, pool, &W, msg));
    if (m) TRY(vec_view(ctx, m, pool, &Mv, msg));
    NewCsr r;
    TRY(write_step(ctx, W, T, m ? &Mv : nullptr, desc, accum, pool, &r, msg));
    TRY(install_vector(ctx, w, r, msg));
    return lagr_ok(msg);
}

static int ewise(bool uni, lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_binop op,
                 const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg)
{
    if (!C || !A || !B || !ctx) return lagr_fail(msg, LAGR_NULL_POINTER, "NULL argument");
    TRY(check_desc(desc, msg));
    if ((int)op <= 0 || (int)op > (int)LAGR_ANY) return lagr_fail(msg, LAGR_INVALID_VALUE, "unknown operator");
    const bool t0 = desc & LAGR_DESC_TRAN0, t1 = desc & LAGR_DESC_TRAN1;
    const int64_t ar = t0 ? A->ncols : A->nrows, ac = t0 ? A->nrows : A->ncols;
    const int64_t br = t1 ? B->ncols : B->nrows, bc = t1 ? B->nrows : B->ncols;
    if (ar != br || ac != bc || C->nrows != ar || C->ncols != ac)
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "operand dimensions differ");
    if (M && (M->nrows != C->nrows || M->ncols != C->ncols))
        return lagr_fail(msg, LAGR_DIMENSION_MISMATCH, "mask dimensions differ from C");
    if (C->type == LAGR_BOOL) return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "eWise needs a valued output");
    if (op == LAGR_DIV && C->type != LAGR_FP64)
        return lagr_fail(msg, LAGR_DOMAIN_MISMATCH, "DIV is defined on FP64 only");
    TRY(check_accum(accum, C->type, msg));
    Pool pool(ctx);
    Csr A2 = view(A), B2 = view(B);
    if (t0) TRY(cached_transpose(ctx, A, &A2, msg));
    if (t1) TRY(cached_transpose(ctx, B, &B2, msg));
    const int vk = vkind_of(C->type);
    int64_t *off = (int64_t *)pool.get(8 * (ar + 1));
    if (!off) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "ewise");
    TRY(fill_i64(ctx, off + ar, 1, 0, msg));
    if (ar > 0) {
        if (uni)
            hipLaunchKernelGGL(k_ewise<true>, G1(ar), A2, B2, (int)op, vk, vkind_of(A->type),
                               vkind_of(B->type), (const int64_t *)nullptr, off, (int32_t *)nullptr,
                               (uint64_t *)nullptr);
        else
            hipLaunchKernelGGL(k_ewise<false>, G1(ar), A2, B2, (int)op, vk, vkind_of(A->type),
                               vkind_of(B->type), (const int64_t *)nullptr, off, (int32_t *)nullptr,
                               (uint64_t *)nullptr);
        LAUNCH_CHECK();
    }
    int64_t nnz = 0;
    TRY(scan_exclusive_i64(ctx, off, off, ar + 1, &nnz, msg));
    int32_t *ci = (int32_t *)pool.get(4 * (nnz > 0 ? nnz : 1));
    uint64_t *va = (uint64_t *)pool.get(8 * (nnz > 0 ? nnz : 1));
    if (!ci || !va) return lagr_fail(msg, LAGR_OUT_OF_MEMORY, "ewise");
    if (ar > 0) {
        if (uni)
            hipLaunchKernelGGL(k_ewise<true>, G1(ar), A2, B2, (int)op, vk, vkind_of(A->type),
                               vkind_of(B->type), off, (int64_t *)nullptr, ci, va);
        else
            hipLaunchKernelGGL(k_ewise<false>, G1(ar), A2, B2, (int)op, vk, vkind_of(A->type),
                               vkind_of(B->type), off, (int64_t *)nullptr, ci, va);
        LAUNCH_CHECK();
    }
    Csr T;
    T.nrows = ar;
    T.ncols = ac;
    T.nvals = nnz;
    T.rp = off;
    T.ci = ci;
    T.val = va;
    T.type = C->type;
    Csr Mv;
    if (M) Mv = view(M);
    NewCsr r;
    TRY(write_step(ctx, view(C), T, M ? &Mv : nullptr, desc, accum, pool, &r, msg));
    install_matrix(ctx, C, r);
    return lagr_ok(msg);
}

extern "C" int lagr_ewise_add(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_binop op,
                              const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg)
{
    return ewise(true, C, M, accum, op, A, B, desc, ctx, msg);
}

extern "C" int lagr_ewise_mult(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_binop op,
                               const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg)
{
    return ewise(false, C, M, accum, op, A, B, desc, ctx, msg);
}
