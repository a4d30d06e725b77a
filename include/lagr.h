/*
 * lagr.h -- C ABI of a masked-semiring sparse library for one AMD Instinct
 * MI355X (gfx950).
 *
 * The library computes the operations that LAGraph (Szarnyas et al.,
 * arXiv 2104.01661) builds its algorithms from: masked products over a
 * semiring, C<M> accum= A (+).(x) B  (Section III, Table I: mxm, vxm, mxv),
 * with a mask that may be valued or structural and complemented, merge or
 * replace semantics ("Masks"), an optional accumulator, transposes through
 * a descriptor, plus reduce, assign, eWiseAdd/eWiseMult and a strictly
 * lower select.  On top of them sit triangle counting (Section IV-E,
 * Algorithm 6), direction-optimising BFS (Section IV-A, Algorithms 1-2) and
 * batched betweenness centrality (Section IV-B, Algorithm 3), a batched
 * many-graph triangle count and a continuous-batching query server.
 *
 * Conventions (Section II, "Algorithm calling conventions", "Error
 * handling"):
 *  - Every call returns int: 0 success, > 0 warning, < 0 error.
 *  - The last argument `msg` is a caller-owned char[LAGR_MSG_LEN] (may be
 *    NULL).  On error or warning it holds a reason; on success it is set to
 *    the empty string.
 *  - Outputs come first and are passed by pointer; the library allocates
 *    them (through the allocator registered with lagr_set_allocator).  A
 *    NULL output pointer means the output is not wanted.
 *  - Input/output objects are passed by value and are modified.
 *  - Inputs are never modified.  Arrays handed to the *_wrap_* calls are
 *    BORROWED device pointers: the caller keeps them alive and unchanged
 *    while the object that wraps them is in use.  When an operation writes
 *    a wrapped object it replaces the borrowed arrays with library-owned
 *    ones and never writes or frees the caller's memory.
 *  - Arguments are validated on the host before any device work; a failed
 *    validation leaves every object unchanged.
 *  - Execution is non-blocking (the GraphBLAS non-blocking mode the paper
 *    relies on for fusion, Section VI-B): device work is queued on the
 *    context's stream.  Results held in device objects are valid once
 *    lagr_wait(ctx) returns or the stream is synchronised; a call whose
 *    output is a host scalar synchronises before it returns.  Temporary
 *    buffers and replaced arrays are freed when the context next waits for
 *    its stream, never by a wait of their own.  Apart from host scalars, a
 *    call waits only to read back a size that it must know on the host to
 *    allocate: the entry count of a CSR result, or of a vector operand
 *    that it turns into a list.  The BFS-shaped vxm calls never wait.
 *  - A transpose descriptor (TRAN0 / TRAN1) uses the matrix's transpose,
 *    built by the first call that needs it and kept with the matrix until
 *    its arrays change; a wrapped matrix whose borrowed arrays the caller
 *    changes must be wrapped again.
 *  - One context per host thread.  Objects may be read by several calls at
 *    once but not written by two at once.
 *
 * Storage:
 *  - lagr_matrix: compressed sparse row (CSR) -- int64 row offsets
 *    (nrows+1), int32 column ids sorted ascending and unique in each row,
 *    optional values (one int64 or double per entry; none for LAGR_BOOL,
 *    whose entries all have the value 1).
 *  - lagr_vector: SPARSE (int32 ids sorted ascending + values), BITMAP
 *    (uint8 presence[n] + dense values[n]) or FULL (dense values, every
 *    entry present).
 */
#ifndef LAGR_H
#define LAGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAGR_MSG_LEN 256

/* ---------------------------------------------------------------- codes */
enum {
    LAGR_SUCCESS = 0,
    LAGR_NO_VALUE = 1,            /* warning: a reduction had no entry     */
    LAGR_NULL_POINTER = -1,
    LAGR_INVALID_VALUE = -2,
    LAGR_INVALID_INDEX = -3,
    LAGR_DOMAIN_MISMATCH = -4,
    LAGR_DIMENSION_MISMATCH = -5,
    LAGR_INVALID_OBJECT = -6,     /* lagr_graph_check found a bad matrix   */
    LAGR_OUT_OF_MEMORY = -7,
    LAGR_PROPERTY_MISSING = -8,   /* an Advanced-mode call lacks a cached property */
    LAGR_NOT_IMPLEMENTED = -9,
    LAGR_DEVICE_ERROR = -10,      /* HIP error; its text is in msg         */
    LAGR_BUDGET_EXCEEDED = -11    /* server: query larger than the budget  */
};

/* Run an lagr call; on error jump to the user-defined LAGR_CATCH (Section
 * II, "Error handling").  Warnings (> 0) are not errors. */
#define LAGR_TRY(call)                         \
    do {                                       \
        int lagr_status_ = (call);             \
        if (lagr_status_ < 0) {                \
            LAGR_CATCH(lagr_status_);          \
        }                                      \
    } while (0)

/* ---------------------------------------------------------------- enums */
/* LAGR_INT32 arrays that cross the boundary (wraps, extracts, host
 * scalars) hold int32 values.  Inside, every value takes an 8-byte slot, so
 * a wrap of INT32 values copies them (widened) into library-owned storage
 * -- the row offsets and ids stay borrowed -- and arithmetic whose result
 * type is INT32 wraps modulo 2^32, as in the GraphBLAS INT32 domain. */
typedef enum {
    LAGR_BOOL = 0,   /* pattern only; every present entry has the value 1 */
    LAGR_INT64 = 1,
    LAGR_FP64 = 2,
    LAGR_INT32 = 3
} lagr_type;

/* The semirings of Table II that the path uses.  Result domains:
 *   PLUS_PAIR   plus monoid, pair(x,y) = 1         -> INT64 (a count)
 *   ANY_SECONDI any monoid,  secondi(a_ik,b_kj) = k -> INT64 (an index)
 *   PLUS_FIRST  plus monoid, first(x,y) = x         -> the type of A'
 *               (LAGR_BOOL A' gives INT64, LAGR_INT32 gives INT32)
 *   MIN_PLUS    min monoid (identity +inf), x + y   -> FP64
 * The additive identity is never stored: an output entry exists iff at
 * least one k has both A'(i,k) and B'(k,j).  The `any` monoid returns one
 * admissible k; this library always returns the smallest, so results are
 * reproducible (LAGR_DESC_DETERMINISTIC states that guarantee).  FP64 sums
 * are taken in ascending k order, except where a call documents otherwise. */
typedef enum {
    LAGR_PLUS_PAIR = 0,
    LAGR_ANY_SECONDI = 1,
    LAGR_PLUS_FIRST = 2,
    LAGR_MIN_PLUS = 3
} lagr_semiring;

/* Binary operators for accumulators, eWise operations and reductions.
 * LAGR_NOOP as an accumulator means "no accumulator". FIRST(c,t)=c,
 * SECOND(c,t)=t, ANY(c,t)=c, DIV is FP64 only. */
typedef enum {
    LAGR_NOOP = 0,
    LAGR_PLUS = 1,
    LAGR_MIN = 2,
    LAGR_FIRST = 3,
    LAGR_SECOND = 4,
    LAGR_TIMES = 5,
    LAGR_DIV = 6,
    LAGR_ANY = 7
} lagr_binop;

/* Descriptor bits (Table I caption; Section III "Masks"). */
#define LAGR_DESC_DEFAULT 0u
#define LAGR_DESC_COMP 1u          /* complement the mask                  */
#define LAGR_DESC_STRUCT 2u        /* structural mask: presence only       */
#define LAGR_DESC_REPLACE 4u       /* delete output entries outside mask   */
#define LAGR_DESC_TRAN0 8u         /* use the transpose of the first input */
#define LAGR_DESC_TRAN1 16u        /* use the transpose of the second input*/
#define LAGR_DESC_DETERMINISTIC 32u/* any monoid returns the smallest k    */
#define LAGR_DESC_ASSIGN_PARENT 64u/* vxm only: also m<s(w)> = w (fused)   */
#define LAGR_DESC_S (LAGR_DESC_STRUCT)
#define LAGR_DESC_RSC (LAGR_DESC_REPLACE | LAGR_DESC_STRUCT | LAGR_DESC_COMP)

typedef enum { LAGR_VEC_SPARSE = 0, LAGR_VEC_BITMAP = 1, LAGR_VEC_FULL = 2 } lagr_vformat;

/* Graph kinds (Listing 1, LAGraph_Kind). */
typedef enum { LAGR_ADJACENCY_UNDIRECTED = 0, LAGR_ADJACENCY_DIRECTED = 1 } lagr_kind;

typedef struct lagr_ctx_s *lagr_ctx;
typedef struct lagr_matrix_s *lagr_matrix;
typedef struct lagr_vector_s *lagr_vector;
typedef struct lagr_graph_s *lagr_graph;

/* ------------------------------------------------------ memory, context */

/* Device allocator used for every library-owned array and workspace
 * (Section V, memory-manager wrappers).  alloc returns NULL on failure,
 * which surfaces as LAGR_OUT_OF_MEMORY.  Passing NULLs restores the
 * built-in hipMalloc/hipFree.  Must be called while no object allocated by
 * the previous allocator is still alive. */
typedef void *(*lagr_alloc_fn)(size_t bytes, void *user);
typedef void (*lagr_free_fn)(void *ptr, size_t bytes, void *user);
int lagr_set_allocator(lagr_alloc_fn alloc, lagr_free_fn release, void *user, char *msg);

/* A context binds a device and a stream (a hipStream_t, NULL = the null
 * stream) and owns a reusable workspace, so repeated calls do not allocate
 * (the per-call allocation cost the paper blames for the high-diameter
 * Road graph, Section VI-B). */
int lagr_ctx_new(lagr_ctx *ctx, int device, void *stream, char *msg);
/* device = -1 makes a validation-only context: every call checks its
 * arguments exactly as usual, but no device work can run on it (calls that
 * pass their checks fail with LAGR_DEVICE_ERROR or LAGR_OUT_OF_MEMORY).  It
 * needs no GPU, so host-side tests of the argument checks can use it. */
/* Switch the context's stream; work queued on the old stream finishes
 * first (the call waits for it). */
int lagr_ctx_set_stream(lagr_ctx ctx, void *stream, char *msg);
int lagr_ctx_free(lagr_ctx *ctx);
/* Wait for all work queued on the context's stream. */
int lagr_wait(lagr_ctx ctx, char *msg);
/* Kernel timing (Section V, Tic/Toc): while enabled, the library brackets
 * each launch of its main kernels with HIP events on the context's stream.
 * lagr_ctx_kernel_time synchronises and returns the summed duration (ms)
 * and launch count of the kernel named `kernel` (e.g. "tc_rows",
 * "bfs_push", "bfs_pull", "bc_forward", "bc_backward") since the timer was
 * last enabled; enabling again clears the record. */
int lagr_ctx_timing(lagr_ctx ctx, int enable, char *msg);
int lagr_ctx_kernel_time(lagr_ctx ctx, const char *kernel, double *total_ms, int64_t *launches,
                         char *msg);

/* ------------------------------------------------------------ matrices */

/* An empty nrows x ncols CSR matrix of the given type. */
int lagr_matrix_new(lagr_matrix *A, lagr_type type, int64_t nrows, int64_t ncols,
                    lagr_ctx ctx, char *msg);
/* Wrap caller device arrays as a CSR matrix (borrowed; see above).
 * rowptr: int64[nrows+1], rowptr[0] = 0, rowptr[nrows] = nvals;
 * colidx: int32[nvals]; values: int64, double or int32 [nvals] by type,
 * NULL for BOOL.
 * Sortedness is the caller's promise; lagr_graph_check verifies it. */
int lagr_matrix_wrap_csr(lagr_matrix *A, lagr_type type, int64_t nrows, int64_t ncols,
                         int64_t nvals, const int64_t *rowptr, const int32_t *colidx,
                         const void *values, lagr_ctx ctx, char *msg);
/* Matrix build from tuples (Table I, build), on the device: nedges pairs
 * (src[e], dst[e]) of int32 device arrays.  flags: LAGR_BUILD_SYMMETRIZE
 * adds (dst, src) for every pair, LAGR_BUILD_DROP_LOOPS drops i == j.
 * Duplicates collapse to one entry.  The result is a LAGR_BOOL CSR. */
#define LAGR_BUILD_SYMMETRIZE 1u
#define LAGR_BUILD_DROP_LOOPS 2u
int lagr_matrix_build(lagr_matrix *A, int64_t nrows, int64_t ncols, int64_t nedges,
                      const int32_t *src, const int32_t *dst, uint32_t flags,
                      lagr_ctx ctx, char *msg);
int lagr_matrix_info(const lagr_matrix A, lagr_type *type, int64_t *nrows, int64_t *ncols,
                     int64_t *nvals, char *msg);
/* Copy A's arrays into caller device buffers of sizes nrows+1 / nvals /
 * nvals (any pointer may be NULL to skip that array). */
int lagr_matrix_extract_csr(const lagr_matrix A, int64_t *rowptr, int32_t *colidx,
                            void *values, lagr_ctx ctx, char *msg);
/* C = strictly lower part of A: entries (i, j) with j < i (Table I,
 * select; the reading of Algorithm 6's tril as strictly lower). */
int lagr_select_tril(lagr_matrix *C, const lagr_matrix A, lagr_ctx ctx, char *msg);
int lagr_matrix_free(lagr_matrix *A);

/* ------------------------------------------------------------- vectors */
int lagr_vector_new(lagr_vector *v, lagr_type type, int64_t n, lagr_ctx ctx, char *msg);
/* Borrowed wraps.  idx int32[nvals] sorted ascending; present uint8[n]
 * (0 / 1); values int64, double or int32 arrays by type (NULL for BOOL). */
int lagr_vector_wrap_sparse(lagr_vector *v, lagr_type type, int64_t n, int64_t nvals,
                            const int32_t *idx, const void *values, lagr_ctx ctx, char *msg);
int lagr_vector_wrap_bitmap(lagr_vector *v, lagr_type type, int64_t n, const uint8_t *present,
                            const void *values, lagr_ctx ctx, char *msg);
int lagr_vector_wrap_full(lagr_vector *v, lagr_type type, int64_t n, const void *values,
                          lagr_ctx ctx, char *msg);
int lagr_vector_info(const lagr_vector v, lagr_type *type, int64_t *n, lagr_vformat *format,
                     char *msg);
/* Number of entries (Table I, nvals); synchronises. */
int lagr_vector_nvals(int64_t *nvals, const lagr_vector v, lagr_ctx ctx, char *msg);
int lagr_matrix_nvals(int64_t *nvals, const lagr_matrix A, lagr_ctx ctx, char *msg);
/* Tuples of v (Table I, extractTuples) into caller device buffers of
 * length nvals (idx ascending). */
int lagr_vector_extract_tuples(const lagr_vector v, int32_t *idx, void *values, lagr_ctx ctx,
                               char *msg);
/* Dense copy: present uint8[n] (may be NULL) and values[n] (absent
 * entries are left as `fill`, a pointer to one element of v's type, or 0
 * when fill is NULL). */
int lagr_vector_extract_dense(const lagr_vector v, uint8_t *present, void *values,
                              const void *fill, lagr_ctx ctx, char *msg);
int lagr_vector_free(lagr_vector *v);

/* --------------------------------------------------- core operations */

/* C<M> accum= A' (+).(x) B'   (Table I, mxm; Section III "Masks").
 * A' = A or A^T (LAGR_DESC_TRAN0), B' = B or B^T (LAGR_DESC_TRAN1).
 * Dimensions: A' m x k, B' k x n, C and M m x n.  M may be NULL (no mask).
 * accum: LAGR_NOOP or a binop on C's type.  C's type must equal the
 * semiring's result type.  C may be the same object as A, B or M; the
 * result is computed into new storage before C is replaced.
 * With a mask that is not complemented the product is computed in dot
 * form, entry by entry on the mask's pattern, from rows of A' and rows of
 * B'^T -- under LAGR_DESC_TRAN1 those are B's own rows, so Algorithm 6's
 * C<s(L)> = L plus.pair L^T reads L twice and transposes nothing;
 * plus.pair there runs the triangle-count intersection kernels.  Other
 * shapes run in saxpy form over rows of B'. */
int lagr_mxm(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_semiring semiring,
             const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg);

/* w'<m'> accum= u' (+).(x) A'  (Table I, vxm; with LAGR_DESC_TRAN1 it is
 * the pull form w<m> accum= A (+).(x) u of mxv).  u length m, A' m x n,
 * w and m length n.
 * LAGR_DESC_ASSIGN_PARENT (an extension: the fused vxm + assign of BFS,
 * Section VI-B) makes the mask the parent vector p of Algorithms 1-2: m
 * must be INT64 and receives m<s(w)> = w after the product (m is then an
 * inout argument and may change storage format).
 * Execution: the BFS-shaped calls -- any.secondi, accum NOOP, a mask with
 * LAGR_DESC_RSC (push over A, or pull over the stored AT with TRAN1),
 * with or without ASSIGN_PARENT -- run on dedicated kernels that enqueue
 * on ctx's stream and return without waiting: w becomes a bitmap vector
 * whose entry count stays on the device (lagr_vector_nvals reads that one
 * word), and its arrays are double-buffered by ctx, so a loop such as
 * q<!s(p), r> = q any.secondi A allocates nothing after its first steps.
 * Push and pull give the same w (the smallest admissible k).  Every other
 * shape is computed on the general path, which waits for the stream. */
int lagr_vxm(lagr_vector w, const lagr_vector m, lagr_binop accum, lagr_semiring semiring,
             const lagr_vector u, const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg);

/* Fused product and reduction: *s = plus-reduce of (C<M> = A' (+).(x) B'),
 * without forming C (Section VI-B, the mxm + reduce fusion proposed for
 * triangle counting).  The result is written to the host scalar *s (int64
 * or double by the semiring's result type); synchronises. */
int lagr_mxm_reduce(void *s, const lagr_matrix M, lagr_semiring semiring, const lagr_matrix A,
                    const lagr_matrix B, uint32_t desc, lagr_ctx ctx, char *msg);

/* s accum= reduce of every entry of A with `monoid` (LAGR_PLUS or
 * LAGR_MIN) (Table I, reduce to scalar).  s is a host scalar of A's type
 * (int64 for BOOL, int32 for INT32).  No entry: s is left unchanged and LAGR_NO_VALUE is
 * returned.  Entries are combined in row-major order.  Synchronises. */
int lagr_reduce_scalar(void *s, lagr_binop accum, lagr_binop monoid, const lagr_matrix A,
                       lagr_ctx ctx, char *msg);
int lagr_vector_reduce_scalar(void *s, lagr_binop accum, lagr_binop monoid, const lagr_vector u,
                              lagr_ctx ctx, char *msg);
/* w<m> accum= row-wise reduce of A' (Table I, reduce to vector); with
 * LAGR_DESC_TRAN0, A' = A^T, i.e. column sums.  Empty rows give no entry. */
int lagr_reduce_rows(lagr_vector w, const lagr_vector m, lagr_binop accum, lagr_binop monoid,
                     const lagr_matrix A, uint32_t desc, lagr_ctx ctx, char *msg);

/* w<m>(:) accum= u  and  w<m>(:) accum= s  (Table I, assign; all indices;
 * s points to one host value of w's type). */
int lagr_assign_vector(lagr_vector w, const lagr_vector m, lagr_binop accum, const lagr_vector u,
                       uint32_t desc, lagr_ctx ctx, char *msg);
int lagr_assign_scalar(lagr_vector w, const lagr_vector m, lagr_binop accum, const void *s,
                       uint32_t desc, lagr_ctx ctx, char *msg);

/* C<M> accum= A op B on the union (eWiseAdd) or intersection (eWiseMult)
 * of the patterns (Table I). */
int lagr_ewise_add(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_binop op,
                   const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx,
                   char *msg);
int lagr_ewise_mult(lagr_matrix C, const lagr_matrix M, lagr_binop accum, lagr_binop op,
                    const lagr_matrix A, const lagr_matrix B, uint32_t desc, lagr_ctx ctx,
                    char *msg);

/* -------------------------------------------------------------- graphs */

/* Move constructor (Listing 1, LAGraph_New): G takes ownership of *A and
 * *A becomes NULL.  A must be square. */
int lagr_graph_new(lagr_graph *G, lagr_matrix *A, lagr_kind kind, lagr_ctx ctx, char *msg);
/* CheckGraph (Section V): rows sorted and unique, ids in range, and for an
 * undirected graph a symmetric pattern.  Records ndiag (Listing 1).
 * LAGR_INVALID_OBJECT with the reason in msg when a check fails. */
int lagr_graph_check(lagr_graph G, lagr_ctx ctx, char *msg);
/* Cached properties (Section V, Property_*): computed and kept in G. */
int lagr_property_row_degree(lagr_graph G, lagr_ctx ctx, char *msg);
/* The triangle-count operand: A relabelled by descending degree and its
 * strictly lower part (Algorithm 6, the degree sort and L = tril(A)). */
int lagr_property_tc_lower(lagr_graph G, lagr_ctx ctx, char *msg);
/* Cached transpose AT of a directed graph's adjacency matrix (Section II,
 * the AT property that pull steps need: row v of AT lists the in-edges of
 * v, with their values).  A no-op for an undirected graph, whose A is its
 * own transpose.  lagr_bfs and lagr_bc compute it on first use for a
 * directed graph; lagr_graph_delete_properties frees it. */
int lagr_property_at(lagr_graph G, lagr_ctx ctx, char *msg);
/* Drop the cached property arrays -- row degree and the triangle-count
 * operand (Section V, DeleteProperties).  The results of lagr_graph_check
 * (ndiag, symmetry) describe A, which a graph never changes, and are kept. */
int lagr_graph_delete_properties(lagr_graph G, lagr_ctx ctx, char *msg);
/* Tuning settings kept in G (lagr_graph_delete_properties keeps them):
 * tc_hubs, the count plan's hub columns (-1: the default, n/256 capped at
 * 4,096 from 2^18 vertices on, else none; changing it drops the cached
 * triangle-count operand, after
 * waiting for ctx's stream), and the BFS direction thresholds alpha and
 * beta (> 0; -1 keeps the current value).  Other values fail with
 * LAGR_INVALID_VALUE.  lagr_graph_get_tuning reads the three back (NULL
 * pointers are skipped).  lagr_tc_autotune and lagr_bfs_autotune set them
 * by timing. */
int lagr_graph_set_tuning(lagr_graph G, int64_t tc_hubs, int32_t bfs_alpha, int32_t bfs_beta, lagr_ctx ctx,
                          char *msg);
int lagr_graph_get_tuning(int64_t *tc_hubs, int32_t *bfs_alpha, int32_t *bfs_beta, const lagr_graph G, char *msg);
/* Borrowed read access to G->A and to the cached triangle-count operand
 * (NULL if not computed).  The handles stay owned by G: do not free them. */
int lagr_graph_matrix(lagr_matrix *A, const lagr_graph G, char *msg);
int lagr_graph_tc_lower(lagr_matrix *L, const lagr_graph G, char *msg);
/* Borrowed handle of AT (G's own A for an undirected graph);
 * LAGR_PROPERTY_MISSING for a directed graph before lagr_property_at. */
int lagr_graph_at(lagr_matrix *AT, const lagr_graph G, char *msg);
int lagr_graph_ndiag(int64_t *ndiag, const lagr_graph G, char *msg);
int lagr_graph_free(lagr_graph *G);

/* ---------------------------------------------------------- algorithms */

/* Triangle count (Section IV-E, Algorithm 6), Basic mode: computes any
 * missing property (requires an undirected graph with no self-loops) and
 * returns the plus-reduction of C<s(L)> = L plus.pair L^T over the
 * degree-ordered strictly lower part L.  `method` picks how:
 *   LAGR_TC_DEFAULT  the count plan of lagr_tc_adv (each pair of L's rows
 *                    intersected once on its cheaper side, C never formed);
 *   LAGR_TC_DOT      the fused masked dot of lagr_mxm_reduce over L (the
 *                    mxm + reduce fusion of Section VI-B, no plan);
 *   LAGR_TC_MXM      Algorithm 6 as written: C formed by lagr_mxm, then
 *                    lagr_reduce_scalar (the unfused form).
 * All give the same count; another method is LAGR_INVALID_VALUE.
 * Synchronises. */
#define LAGR_TC_DEFAULT 0
#define LAGR_TC_DOT 1
#define LAGR_TC_MXM 2
int lagr_tc(int64_t *ntriangles, lagr_graph G, int method, lagr_ctx ctx, char *msg);
/* Advanced mode (Section II, "User modes"): LAGR_PROPERTY_MISSING when
 * lagr_property_tc_lower has not been computed; never computes it. */
int lagr_tc_adv(int64_t *ntriangles, const lagr_graph G, lagr_ctx ctx, char *msg);
/* Allocation-free variant of lagr_tc_adv, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  It calls no allocator and does not synchronise:
 * the count is written to ntriangles_dev, a DEVICE int64 owned by the
 * caller, valid once ctx's stream has reached that point.  The workgroup
 * partials and work counters live in a fixed per-device scratch array of
 * the library (4,096 partials + 129 words, 33.8 KB, held until the process
 * ends); a grid that would need more partials is rejected with
 * LAGR_INVALID_VALUE before any launch.  Every call on one GPU shares that
 * scratch: calls that overlap on one GPU (two streams, two threads) race
 * and must be serialised by the caller.  LAGR_PROPERTY_MISSING when
 * lagr_property_tc_lower has not been computed. */
int lagr_tc_adv_noalloc(int64_t *ntriangles_dev, const lagr_graph G, lagr_ctx ctx, char *msg);

/* The count plan's hub columns of G, picked by timing: each candidate
 * (none, or n/1024 .. n/128 of the highest-degree vertices, at most 4,096)
 * rebuilds the triangle-count preparation and times lagr_tc (median of 3);
 * the fastest is kept in G (it survives lagr_graph_delete_properties) and
 * the operand is left built.  hubs (may be NULL): the chosen count.  Every
 * candidate must give the same count (else LAGR_DEVICE_ERROR). */
int lagr_tc_autotune(int64_t *hubs, lagr_graph G, lagr_ctx ctx, char *msg);

/* Breadth-first search (Section IV-A, Algorithms 1-2).  Outputs (either
 * may be NULL): level, an INT64 FULL vector (source 0, -1 unreached) and
 * parent, an INT64 FULL vector (parent(src) = src, -1 unreached).  Each
 * level is a fused any.secondi step under the complemented structural mask
 * of visited vertices, written straight into parent: push over the
 * frontier list, or pull over unvisited vertices with a frontier bitmap
 * when the frontier's edges outweigh the unexplored ones (Beamer's
 * heuristic).  Parents are the smallest valid parent unless
 * LAGR_BFS_ANY_PARENT allows any valid one.  On a directed graph the search
 * follows out-edges (A(u, v) is u -> v) and the parent of v is an
 * in-neighbour; pull steps read AT, which is computed and cached on first
 * use unless LAGR_BFS_PUSH_ONLY is given.  The call returns once the
 * search has ended (it watches a word the device stores when a level finds
 * the frontier empty), possibly before the last few queued level kernels,
 * which only pass the finished state on, have run: the outputs are valid
 * after lagr_wait or a sync of the context's stream, like every device
 * output. */
#define LAGR_BFS_PUSH_ONLY 1u
#define LAGR_BFS_ANY_PARENT 2u
int lagr_bfs(lagr_vector *level, lagr_vector *parent, const lagr_graph G, int64_t source,
             uint32_t flags, lagr_ctx ctx, char *msg);

/* BFS direction thresholds of G, picked by timing lagr_bfs from the HOST
 * int64 sources[ns] (total over the sources) for alpha in {6, 10, 14, 20,
 * 32} x beta in {12, 24, 48}: a level pulls when its frontier's edges
 * exceed the unexplored edges / alpha and pushes again below n / beta
 * frontier vertices.  The pair is kept in G for later searches (levels and
 * default parents do not depend on it); alpha, beta (may be NULL) return
 * it. */
int lagr_bfs_autotune(int32_t *alpha, int32_t *beta, lagr_graph G, const int64_t *sources, int32_t ns,
                      lagr_ctx ctx, char *msg);

/* Breadth-first search from many sources at once: Algorithm 1 with a
 * matrix frontier, Q<!s(P), r> = Q any.secondi A for a block of up to 64
 * sources (one wavefront lane each, 64-bit lane masks per vertex), push or
 * pull per level as lagr_bfs chooses.  The start and the first 8 levels of
 * each block replay one captured hipGraph; the level directions and the end
 * are decided on the device.  sources: HOST int64[ns] (repeats allowed).
 * Outputs (each may be NULL): levels, a caller-owned DEVICE int32 array of
 * ns x n (row k: the level of every vertex from sources[k], -1 unreached);
 * reached, level_sum, depth: caller-owned HOST int64 arrays of ns (vertices
 * reached with the source, the sum of their levels, the largest level).
 * Undirected graphs only (LAGR_INVALID_VALUE otherwise); LAGR_INVALID_INDEX
 * for a source outside [0, n).  Synchronises. */
int lagr_bfs_batch(int32_t *levels, int64_t *reached, int64_t *level_sum, int64_t *depth, const lagr_graph G,
                   const int64_t *sources, int32_t ns, lagr_ctx ctx, char *msg);

/* Batched betweenness centrality (Section IV-B, Algorithm 3): unnormalised
 * sum over the given sources of the dependency of every vertex, where a
 * source contributes nothing to itself.  `sources` is a HOST int64 array;
 * they are processed in batches of 64 (one source per wavefront lane) and
 * the batches are summed in order.  Output: FP64 FULL vector.  On a directed
 * graph shortest paths follow out-edges; pull steps read AT, which is
 * computed and cached on first use. */
int lagr_bc(lagr_vector *centrality, const lagr_graph G, const int64_t *sources, int32_t ns,
            lagr_ctx ctx, char *msg);
/* lagr_bc with a choice for the backward sweep (Section IV-B gives both
 * forms of its step: pull W = W A^T, push W = W B).  flags 0: pull on every
 * level, which adds each vertex's terms in a fixed order, so the result is
 * the same bits on every run (what lagr_bc does).
 * LAGR_BC_BACKWARD_PUSH_PULL: push where level i has fewer edges than
 * level i-1 / 4, else pull; LAGR_BC_BACKWARD_PUSH_ONLY: push on every
 * level.  Push adds with FP64 atomics in no fixed order: the scores then
 * agree with the pull's to rounding (relative differences of a few ulps
 * per level), not bit for bit.  Other flags: LAGR_INVALID_VALUE. */
#define LAGR_BC_BACKWARD_PUSH_PULL 1u
#define LAGR_BC_BACKWARD_PUSH_ONLY 2u
int lagr_bc_dir(lagr_vector *centrality, const lagr_graph G, const int64_t *sources, int32_t ns,
                uint32_t flags, lagr_ctx ctx, char *msg);

/* Single-source shortest paths by delta-stepping (Section IV-D, Algorithm
 * 5) over the min.plus semiring.  G->A must be LAGR_FP64: A(u, v) is the
 * weight of the edge u -> v (rows are out-edges; any graph kind), and every
 * weight must be positive and finite (Algorithm 5's split into light edges,
 * 0 < w <= delta, and heavy edges, w > delta, has no place for others):
 * LAGR_DOMAIN_MISMATCH for another type, LAGR_INVALID_VALUE for a bad
 * weight or a delta that is not positive and finite, LAGR_INVALID_INDEX
 * for a source outside [0, n).  Output: dist, a new FP64 FULL vector of
 * shortest-path lengths (0 at the source, +inf where unreachable).  Each
 * distance is the minimum over the relaxations made of dist(u) + w(u, v)
 * with the final dist(u) among them, so it equals Dijkstra's result bit for
 * bit for any positive weights. */
int lagr_sssp(lagr_vector *dist, const lagr_graph G, int64_t source, double delta, lagr_ctx ctx,
              char *msg);

/* PageRank as GAP specifies it (Section IV-C, Algorithm 4), in FP64:
 * teleport = (1 - damping)/n, r = 1/n, and each iteration
 * r = teleport + sum over the in-edges i -> j of r_prev(i) / (d_out(i) /
 * damping), where a vertex without out-edges sends nothing (GAP's variant:
 * their rank leaks).  Stops after the first iteration whose change has
 * 1-norm below tol, or after itermax iterations.  damping in [0, 1], tol
 * finite and >= 0, itermax >= 0, else LAGR_INVALID_VALUE.  A directed
 * graph's in-edges are the rows of AT (computed and cached on first use).
 * Output: rank, a new FP64 FULL vector; iters (may be NULL): the
 * iterations run.  Sums over at most 32 in-edges run in ascending order as
 * the listing adds them; longer ones in a fixed order of their own, so a
 * run is reproducible bit for bit. */
int lagr_pagerank(lagr_vector *rank, int64_t *iters, const lagr_graph G, double damping, double tol,
                  int64_t itermax, lagr_ctx ctx, char *msg);

/* Connected components by FastSV (Section IV-F, Algorithm 7): component,
 * a new INT64 FULL vector holding for every vertex the smallest vertex id of
 * its component (weakly connected for a directed graph, whose AT is
 * computed and cached on first use); iters (may be NULL): the FastSV
 * iterations run. */
int lagr_cc(lagr_vector *component, int64_t *iters, const lagr_graph G, lagr_ctx ctx, char *msg);

/* ------------------------------------------------- many-graph batching */

/* Triangle counts of many independent graphs in one launch (an extension
 * of Algorithm 6 beyond the paper: the per-call overhead it blames for
 * small problems, Section VI-B, is paid once for the whole batch).
 * lagr_batch_new computes each graph's missing triangle-count operand and
 * count plan (Basic mode) and packs them back to back on the device (int32
 * local column ids); the graphs may be freed afterwards.  A batch holds
 * fewer than 2^31 rows in total. */
typedef struct lagr_batch_s *lagr_batch;
typedef struct {
    int32_t blocks_per_cu; /* workgroups of 4 wavefronts per compute unit, 1..16 */
    int32_t row_charge;    /* work items a wavefront takes per grab from the work
                              counters (the grain of the dynamic split), >= 1 */
    int32_t use_graph;     /* capture the launch once into a hipGraph and replay it */
} lagr_tune;
int lagr_batch_new(lagr_batch *B, const lagr_graph *graphs, int64_t ngraphs, lagr_ctx ctx,
                   char *msg);
int lagr_batch_info(const lagr_batch B, int64_t *ngraphs, int64_t *rows, int64_t *entries,
                    char *msg);
/* Times a grid of (blocks_per_cu, row_charge) candidates on this batch and
 * stores the fastest (with use_graph = 1) as the batch's default. */
int lagr_batch_autotune(lagr_tune *best, lagr_batch B, lagr_ctx ctx, char *msg);
/* counts: HOST int64[ngraphs], graph order.  tune may be NULL (the batch's
 * default).  Synchronises. */
int lagr_tc_batched(int64_t *counts, lagr_batch B, const lagr_tune *tune, lagr_ctx ctx,
                    char *msg);
int lagr_batch_free(lagr_batch *B);

/* ------------------------------------------------------------ serving */

/* A continuous-batching query server over resident undirected graphs (an
 * extension beyond the paper: the algorithms of Section IV-A/B and
 * Algorithm 6 answered for a stream of queries).  Worker threads, each
 * with its own HIP stream and workspace, take the oldest query whose
 * arrival time has passed together with every other visible query of the
 * same kind on the same graph: up to max_bfs_batch BFS queries run as one
 * multi-source BFS (one wavefront lane each), up to max_bc_batch BC
 * queries of up to 8 sources run as one 64-lane Algorithm 3 batch, and all
 * visible counts of one graph share one count.  While max_bc_workers
 * workers run BC batches, a free worker takes the oldest visible query of
 * another kind instead, so short queries do not wait behind long ones.
 * Memory: the server accounts, per worker, the larger of the device memory
 * its context and buffers hold from earlier batches (measured after each
 * batch) and its running batch's working-set estimate, plus the kept
 * result vectors.  A batch is admitted only when that total, with its own
 * estimate, fits budget_bytes; when nothing runs and it still does not
 * fit, the workers free their held workspaces first.  A batch whose
 * estimate alone exceeds the budget completes with status
 * LAGR_BUDGET_EXCEEDED.  Every result is the same whatever the batch. */
typedef struct lagr_server_s *lagr_server;
enum { LAGR_QUERY_TC = 0, LAGR_QUERY_BFS = 1, LAGR_QUERY_BC = 2 };
typedef struct {
    int32_t workers;        /* worker threads, 1..16 */
    int32_t max_bfs_batch;  /* 1..64 */
    int32_t max_bc_batch;   /* 1..8 */
    int32_t keep_vectors;   /* keep each BFS level / BC vector for lagr_server_result_vector */
    int64_t budget_bytes;   /* device working-set budget over concurrent batches */
    int32_t max_bc_workers; /* workers that may run BC batches at once (0: workers - 2, at least 1) */
    int32_t pad_;
} lagr_server_config;
typedef struct {
    int32_t kind;           /* LAGR_QUERY_* */
    int32_t graph;          /* index into the server's graphs */
    int32_t nsources;       /* TC 0, BFS 1, BC 1..8 */
    int32_t pad_;
    int64_t sources[8];
    double arrival;         /* server clock (s) at which the query becomes visible */
} lagr_query;
typedef struct {
    int64_t ticket;
    int32_t kind, graph;
    int32_t status;         /* LAGR_SUCCESS or the failing call's code */
    int32_t batch_size;     /* queries answered by the same batch */
    int64_t triangles;      /* TC */
    int64_t reached;        /* BFS: vertices reached, the source included */
    int64_t level_sum;      /* BFS: sum of the levels of reached vertices */
    int64_t depth;          /* BFS: largest level */
    double bc_sum;          /* BC: sum over vertices of the centrality */
    double bc_max;          /* BC: largest centrality */
    double arrival, start, done;   /* server clock (s) */
} lagr_result;
typedef struct {
    int64_t completed;
    int64_t batches[3], queries[3];   /* per LAGR_QUERY_* */
    int64_t rejected;
    int64_t peak_bytes;     /* largest accounted use when a batch was admitted: kept vectors +
                               per worker the larger of its held workspace and its running
                               batch's estimate (at most budget_bytes, unless a batch had to
                               run alone beside kept vectors) */
    int64_t pending;
    int64_t device_peak_bytes;   /* largest device use hipMemGetInfo showed after a batch */
    int64_t held_bytes;          /* accounted use now */
} lagr_server_counts;
/* Builds every graph's cached triangle-count operand and long-row chunk
 * list on ctx's stream (so workers never write a graph), then starts the
 * workers on ctx's device.  The graphs must outlive the server and must
 * not be changed while it runs.  Workers allocate with hipMalloc, never
 * through a registered allocator. */
int lagr_server_new(lagr_server *S, const lagr_graph *graphs, int32_t ngraphs,
                    const lagr_server_config *cfg, lagr_ctx ctx, char *msg);
/* Seconds since the server started. */
int lagr_server_clock(const lagr_server S, double *now, char *msg);
/* Copies the query in; ticket (may be NULL) numbers queries in submission
 * order from 0.  Thread-safe. */
int lagr_server_submit(lagr_server S, const lagr_query *q, int64_t *ticket, char *msg);
/* Moves up to max completed results (completion order) into out. */
int lagr_server_poll(lagr_server S, lagr_result *out, int32_t max, int32_t *n, char *msg);
/* Waits until at least n_completed queries have completed in total, or
 * timeout_s passes (then LAGR_NO_VALUE). */
int lagr_server_wait(lagr_server S, int64_t n_completed, double timeout_s, char *msg);
/* With keep_vectors: hands over the kept result of a completed query (BFS:
 * INT64 FULL levels, -1 unreached; BC: FP64 FULL centrality), allocated
 * through ctx; each ticket's vector can be taken once. */
int lagr_server_result_vector(lagr_server S, int64_t ticket, lagr_vector *v, lagr_ctx ctx,
                              char *msg);
int lagr_server_stats(const lagr_server S, lagr_server_counts *stats, char *msg);
/* Stops the workers after their running batches (queries still pending
 * are dropped) and frees everything the server holds. */
int lagr_server_free(lagr_server *S);

#ifdef __cplusplus
}
#endif
#endif /* LAGR_H */
