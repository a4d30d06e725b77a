/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, single-threaded CPU statement of what the device path
 * computes, written from the paper (LAGraph, arXiv 2104.01661).  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the device library.
 *
 * Every function takes an undirected graph as a sorted, duplicate-free,
 * self-loop-free adjacency (int64 row offsets, int32 neighbour ids) that
 * orc_build makes from raw edge draws.
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Graph construction (Table IV stands in as seeded R-MAT draws): add both
 * directions of every draw, drop self-loops, sort each row, drop
 * duplicates.  colidx must have room for 2*m entries.  Returns nnz.       */
/* ---------------------------------------------------------------------- */

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                  int64_t *rowptr, int32_t *colidx)
{
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!fill) return -1;
    for (int64_t e = 0; e < m; e++) {
        if (src[e] == dst[e]) continue;
        fill[src[e]]++;
        fill[dst[e]]++;
    }
    /* raw row starts (with duplicates) */
    int64_t total = 0;
    for (int64_t v = 0; v < n; v++) {
        const int64_t c = fill[v];
        fill[v] = total;
        total += c;
    }
    fill[n] = total;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!start) { free(fill); return -1; }
    memcpy(start, fill, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < m; e++) {
        const int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        colidx[fill[u]++] = v;
        colidx[fill[v]++] = u;
    }
    /* sort each row and squeeze out duplicates, compacting in place */
    int64_t out = 0;
    rowptr[0] = 0;
    for (int64_t v = 0; v < n; v++) {
        int32_t *row = colidx + start[v];
        const int64_t len = start[v + 1] - start[v];
        qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
        for (int64_t p = 0; p < len; p++) {
            if (p > 0 && row[p] == row[p - 1]) continue;
            colidx[out++] = row[p];
        }
        rowptr[v + 1] = out;
    }
    free(start);
    free(fill);
    return out;
}

/* ---------------------------------------------------------------------- */
/* Triangle counting (Section IV-E, Algorithm 6): the number of 3-cliques.
 * Written from the definition: every triangle u < v < w is counted once,
 * at its smallest edge (u, v), by merging the neighbours of u that come
 * after v with the neighbours of v that come after v.  No relabelling: the
 * count does not depend on vertex order.                                   */
/* ---------------------------------------------------------------------- */

int64_t orc_tc(int64_t n, const int64_t *rp, const int32_t *ci)
{
    int64_t t = 0;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            const int32_t v = ci[p];
            if (v <= u) continue;
            /* w in N(u) with w > v: the entries after position p */
            int64_t a = p + 1, ae = rp[u + 1];
            /* w in N(v) with w > v */
            int64_t b = rp[v], be = rp[v + 1];
            while (b < be && ci[b] <= v) b++;
            while (a < ae && b < be) {
                if (ci[a] < ci[b]) a++;
                else if (ci[a] > ci[b]) b++;
                else { t++; a++; b++; }
            }
        }
    }
    return t;
}

/* Same count restricted to the rows u = u0, u0 + stride, ... below u1:
 * used to time a bounded sample of the full workload. */
int64_t orc_tc_rows(int64_t n, const int64_t *rp, const int32_t *ci, int64_t u0, int64_t u1,
                    int64_t stride)
{
    int64_t t = 0;
    if (u1 > n) u1 = n;
    if (stride < 1) stride = 1;
    for (int64_t u = u0; u < u1; u += stride) {
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            const int32_t v = ci[p];
            if (v <= u) continue;
            int64_t a = p + 1, ae = rp[u + 1];
            int64_t b = rp[v], be = rp[v + 1];
            while (b < be && ci[b] <= v) b++;
            while (a < ae && b < be) {
                if (ci[a] < ci[b]) a++;
                else if (ci[a] > ci[b]) b++;
                else { t++; a++; b++; }
            }
        }
    }
    return t;
}

/*
 * The masked product of Algorithm 6 before its reduction, entry by entry:
 * L is the strictly lower part of A (row i keeps neighbours j < i), and
 * C(i,j) = sum over k of L(i,k) pair L(j,k) = |L_i intersect L_j| for every
 * (i,j) in L.  Outputs L's row offsets (n+1), its column ids and the counts
 * aligned with them; lci and cnt need room for nnz(A)/2 entries.
 */
int64_t orc_tc_lower_counts(int64_t n, const int64_t *rp, const int32_t *ci,
                            int64_t *lrp, int32_t *lci, int64_t *cnt)
{
    int64_t q = 0;
    lrp[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t p = rp[i]; p < rp[i + 1] && ci[p] < i; p++) lci[q++] = ci[p];
        lrp[i + 1] = q;
    }
    for (int64_t i = 0; i < n; i++) {
        for (int64_t p = lrp[i]; p < lrp[i + 1]; p++) {
            const int32_t j = lci[p];
            int64_t a = lrp[i], ae = lrp[i + 1], b = lrp[j], be = lrp[j + 1], c = 0;
            while (a < ae && b < be) {
                if (lci[a] < lci[b]) a++;
                else if (lci[a] > lci[b]) b++;
                else { c++; a++; b++; }
            }
            cnt[p] = c;
        }
    }
    return q;
}

/* ---------------------------------------------------------------------- */
/* Breadth-first search (Section IV-A, Algorithms 1 and 2).  A FIFO queue
 * from the source, scanning neighbours in ascending order.  level(s) = 0,
 * parent(s) = s; the first time v is seen from u, level(v) = level(u)+1 and
 * parent(v) = u.  Unreached vertices get -1 in both.                       */
/* ---------------------------------------------------------------------- */

int orc_bfs(int64_t n, const int64_t *rp, const int32_t *ci, int64_t s,
            int32_t *level, int64_t *parent)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return -1;
    for (int64_t v = 0; v < n; v++) { level[v] = -1; parent[v] = -1; }
    int64_t head = 0, tail = 0;
    level[s] = 0;
    parent[s] = s;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
        const int32_t u = queue[head++];
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            const int32_t v = ci[p];
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                parent[v] = u;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* The deterministic reading of the `any` monoid: given the BFS levels, the
 * parent of a reached v != s is the smallest neighbour one level closer. */
void orc_bfs_min_parent(int64_t n, const int64_t *rp, const int32_t *ci, int64_t s,
                        const int32_t *level, int64_t *parent)
{
    for (int64_t v = 0; v < n; v++) {
        parent[v] = -1;
        if (level[v] < 0) continue;
        if (v == s) { parent[v] = s; continue; }
        for (int64_t p = rp[v]; p < rp[v + 1]; p++) {
            if (level[ci[p]] == level[v] - 1) { parent[v] = ci[p]; break; }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Betweenness centrality (Section IV-B, Algorithm 3): Brandes' method in
 * FP64, one source at a time.  A BFS counts shortest paths sigma; walking
 * the BFS order backwards, every predecessor v of w gains
 * sigma(v)/sigma(w) * (1 + delta(w)).  centrality(w) accumulates delta(w)
 * for every w other than the source.  Sources are summed in the order
 * given.  Returns -2 if a path count reaches 2^53 (it would no longer be an
 * exact integer in FP64), -1 on allocation failure.                        */
/* ---------------------------------------------------------------------- */

int orc_brandes(int64_t n, const int64_t *rp, const int32_t *ci, int64_t ns,
                const int64_t *sources, double *centrality)
{
    double *sigma = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *delta = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!sigma || !delta || !dist || !order) {
        free(sigma); free(delta); free(dist); free(order);
        return -1;
    }
    int rc = 0;
    for (int64_t v = 0; v < n; v++) centrality[v] = 0.0;
    for (int64_t k = 0; k < ns; k++) {
        const int64_t s = sources[k];
        for (int64_t v = 0; v < n; v++) { sigma[v] = 0.0; delta[v] = 0.0; dist[v] = -1; }
        int64_t head = 0, tail = 0;
        sigma[s] = 1.0;
        dist[s] = 0;
        order[tail++] = (int32_t)s;
        while (head < tail) {
            const int32_t u = order[head++];
            for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
                const int32_t v = ci[p];
                if (dist[v] < 0) { dist[v] = dist[u] + 1; order[tail++] = v; }
                if (dist[v] == dist[u] + 1) sigma[v] += sigma[u];
            }
        }
        for (int64_t i = 0; i < tail; i++)
            if (sigma[order[i]] >= 9007199254740992.0) rc = -2;
        for (int64_t i = tail - 1; i >= 0; i--) {
            const int32_t w = order[i];
            for (int64_t p = rp[w]; p < rp[w + 1]; p++) {
                const int32_t v = ci[p];
                if (dist[v] == dist[w] - 1) delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
            }
            if (w != s) centrality[w] += delta[w];
        }
    }
    free(sigma); free(delta); free(dist); free(order);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Directed graphs (LAGRAPH_ADJACENCY_DIRECTED, Section II): A(u, v) is the
 * edge u -> v.  The pull steps of Algorithm 2 and the predecessor sweep of
 * Algorithm 3 read the in-edges of a vertex, which are the rows of the
 * transpose (the cached AT property of Section II).                        */
/* ---------------------------------------------------------------------- */

/* Directed adjacency from raw draws: the pair (src[e], dst[e]) is the edge
 * src -> dst; self-loops dropped, rows sorted, duplicates removed.  Returns
 * nnz, or -1 on allocation failure. */
int64_t orc_build_directed(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           int64_t *rowptr, int32_t *colidx)
{
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill || !start) { free(fill); free(start); return -1; }
    for (int64_t e = 0; e < m; e++)
        if (src[e] != dst[e]) fill[src[e]]++;
    int64_t total = 0;
    for (int64_t v = 0; v < n; v++) {
        const int64_t c = fill[v];
        fill[v] = total;
        start[v] = total;
        total += c;
    }
    start[n] = total;
    for (int64_t e = 0; e < m; e++)
        if (src[e] != dst[e]) colidx[fill[src[e]]++] = dst[e];
    int64_t out = 0;
    rowptr[0] = 0;
    for (int64_t v = 0; v < n; v++) {
        int32_t *row = colidx + start[v];
        const int64_t len = start[v + 1] - start[v];
        qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
        for (int64_t p = 0; p < len; p++) {
            if (p > 0 && row[p] == row[p - 1]) continue;
            colidx[out++] = row[p];
        }
        rowptr[v + 1] = out;
    }
    free(fill);
    free(start);
    return out;
}

/* Transpose of an nrows x ncols CSR by counting sort on the column: the
 * entries of every column, taken in row order, become the row of the
 * transpose (so its rows come out sorted).  perm[q] = the entry of A that
 * lands at position q (to carry values).  Returns 0, -1 on allocation
 * failure. */
int orc_transpose(int64_t nrows, int64_t ncols, const int64_t *rp, const int32_t *ci, int64_t *rpT,
                  int32_t *ciT, int64_t *perm)
{
    int64_t *fill = (int64_t *)calloc((size_t)ncols + 1, sizeof(int64_t));
    if (!fill) return -1;
    for (int64_t p = 0; p < rp[nrows]; p++) fill[ci[p] + 1]++;
    for (int64_t c = 0; c < ncols; c++) fill[c + 1] += fill[c];
    for (int64_t c = 0; c <= ncols; c++) rpT[c] = fill[c];
    for (int64_t u = 0; u < nrows; u++)
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            const int64_t q = fill[ci[p]]++;
            ciT[q] = (int32_t)u;
            perm[q] = p;
        }
    free(fill);
    return 0;
}

/* Brandes' betweenness on a directed graph: the BFS counts shortest paths
 * along out-edges (rows of A); the backward sweep credits every
 * predecessor v of w -- an in-neighbour, a row entry of the transpose --
 * with sigma(v)/sigma(w) * (1 + delta(w)).  Same conventions as
 * orc_brandes. */
int orc_brandes_directed(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rpT,
                         const int32_t *ciT, int64_t ns, const int64_t *sources, double *centrality)
{
    double *sigma = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *delta = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!sigma || !delta || !dist || !order) {
        free(sigma); free(delta); free(dist); free(order);
        return -1;
    }
    int rc = 0;
    for (int64_t v = 0; v < n; v++) centrality[v] = 0.0;
    for (int64_t k = 0; k < ns; k++) {
        const int64_t s = sources[k];
        for (int64_t v = 0; v < n; v++) { sigma[v] = 0.0; delta[v] = 0.0; dist[v] = -1; }
        int64_t head = 0, tail = 0;
        sigma[s] = 1.0;
        dist[s] = 0;
        order[tail++] = (int32_t)s;
        while (head < tail) {
            const int32_t u = order[head++];
            for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
                const int32_t v = ci[p];
                if (dist[v] < 0) { dist[v] = dist[u] + 1; order[tail++] = v; }
                if (dist[v] == dist[u] + 1) sigma[v] += sigma[u];
            }
        }
        for (int64_t i = 0; i < tail; i++)
            if (sigma[order[i]] >= 9007199254740992.0) rc = -2;
        for (int64_t i = tail - 1; i >= 0; i--) {
            const int32_t w = order[i];
            for (int64_t p = rpT[w]; p < rpT[w + 1]; p++) {
                const int32_t v = ciT[p];
                if (dist[v] >= 0 && dist[v] == dist[w] - 1) delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
            }
            if (w != s) centrality[w] += delta[w];
        }
    }
    free(sigma); free(delta); free(dist); free(order);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* PageRank as GAP specifies it (Section IV-C, Algorithm 4), in FP64, the
 * steps in the listing's order:
 *   teleport = (1 - damping) / n;  r = 1/n;  d = d_out / damping
 *   repeat: t = r;  w = t / d (only where d_out > 0: a vertex without
 *   out-edges sends nothing);  r = teleport;  r += AT plus.second w, i.e.
 *   r(j) += w(i) for every edge i -> j, summed over i in ascending order;
 *   t = |t - r|;  stop when sum(t), summed over j in ascending order, is
 *   below tol, or after itermax iterations.
 * rpT/ciT: the transpose (row j lists the in-neighbours i of j); dout[i]:
 * out-degree.  Returns the number of iterations done, -1 on allocation
 * failure.                                                                 */
/* ---------------------------------------------------------------------- */

int64_t orc_pagerank(int64_t n, const int64_t *rpT, const int32_t *ciT, const int64_t *dout, double damping,
                     double tol, int64_t itermax, double *r)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!t || !w || !d) { free(t); free(w); free(d); return -1; }
    const double teleport = (1.0 - damping) / (double)n;
    for (int64_t v = 0; v < n; v++) {
        r[v] = 1.0 / (double)n;
        d[v] = (double)dout[v] / damping;
    }
    int64_t k = 0;
    while (k < itermax) {
        k++;
        for (int64_t v = 0; v < n; v++) t[v] = r[v];
        for (int64_t v = 0; v < n; v++) w[v] = dout[v] > 0 ? t[v] / d[v] : 0.0;
        for (int64_t j = 0; j < n; j++) {
            double s = 0.0;
            for (int64_t p = rpT[j]; p < rpT[j + 1]; p++)
                if (dout[ciT[p]] > 0) s += w[ciT[p]];
            r[j] = teleport + s;
        }
        double sum = 0.0;
        for (int64_t j = 0; j < n; j++) sum += fabs(t[j] - r[j]);
        if (sum < tol) break;
    }
    free(t); free(w); free(d);
    return k;
}

/* ---------------------------------------------------------------------- */
/* Connected components (Section IV-F, Algorithm 7).  FastSV only ever
 * lowers a parent to a smaller id and stops when no grandparent changes,
 * which leaves every vertex pointing at the smallest vertex id of its
 * component; that labelling is written out here directly, by a BFS from
 * each not yet labelled vertex in ascending order.  Edges are taken in both
 * directions (rp/ci and the transpose rpT/ciT; pass A twice for an
 * undirected graph).  Returns 0, -1 on allocation failure.                */
/* ---------------------------------------------------------------------- */

int orc_components(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rpT, const int32_t *ciT,
                   int64_t *label)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return -1;
    for (int64_t v = 0; v < n; v++) label[v] = -1;
    for (int64_t s = 0; s < n; s++) {
        if (label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        label[s] = s;
        queue[tail++] = (int32_t)s;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int side = 0; side < 2; side++) {
                const int64_t *R = side ? rpT : rp;
                const int32_t *C = side ? ciT : ci;
                for (int64_t p = R[u]; p < R[u + 1]; p++)
                    if (label[C[p]] < 0) {
                        label[C[p]] = s;
                        queue[tail++] = C[p];
                    }
            }
        }
    }
    free(queue);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Single-source shortest paths (Section IV-D): the distances that the
 * delta-stepping method of Algorithm 5 computes, here by Dijkstra's
 * algorithm with a binary heap of (distance, vertex) pairs (stale pairs are
 * skipped).  Weights w[p] >= 0 belong to CSR entry p.  dist = +inf for
 * unreachable vertices.  Returns 0, or -1 if memory runs out.            */
/* ---------------------------------------------------------------------- */

typedef struct {
    double d;
    int64_t v;
} orc_hnode;

static void orc_heap_push(orc_hnode *h, int64_t *sz, double d, int64_t v)
{
    int64_t i = (*sz)++;
    while (i > 0) {
        const int64_t parent = (i - 1) / 2;
        if (h[parent].d <= d) break;
        h[i] = h[parent];
        i = parent;
    }
    h[i].d = d;
    h[i].v = v;
}

static orc_hnode orc_heap_pop(orc_hnode *h, int64_t *sz)
{
    const orc_hnode top = h[0];
    const orc_hnode last = h[--(*sz)];
    int64_t i = 0;
    while (1) {
        int64_t c = 2 * i + 1;
        if (c >= *sz) break;
        if (c + 1 < *sz && h[c + 1].d < h[c].d) c++;
        if (h[c].d >= last.d) break;
        h[i] = h[c];
        i = c;
    }
    if (*sz > 0) h[i] = last;
    return top;
}

int orc_dijkstra(int64_t n, const int64_t *rp, const int32_t *ci, const double *w, int64_t s, double *dist)
{
    const int64_t cap = rp[n] + 1;
    orc_hnode *h = (orc_hnode *)malloc(sizeof(orc_hnode) * (size_t)cap);
    char *done = (char *)calloc((size_t)n + 1, 1);
    if (!h || !done) {
        free(h);
        free(done);
        return -1;
    }
    for (int64_t v = 0; v < n; v++) dist[v] = 1.0 / 0.0;
    int64_t sz = 0;
    dist[s] = 0.0;
    orc_heap_push(h, &sz, 0.0, s);
    while (sz > 0) {
        const orc_hnode x = orc_heap_pop(h, &sz);
        if (done[x.v]) continue;
        done[x.v] = 1;
        for (int64_t p = rp[x.v]; p < rp[x.v + 1]; p++) {
            const int64_t v = ci[p];
            const double nd = x.d + w[p];
            if (nd < dist[v]) {
                dist[v] = nd;
                orc_heap_push(h, &sz, nd, v);
            }
        }
    }
    free(h);
    free(done);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Timing drivers.  They call the functions above, unchanged, over
 * independent units of work: rows of the triangle count, BFS sources,
 * contiguous ranges of betweenness sources.  Built with OpenMP (the timing
 * build of this same file) the units run on several threads; built without
 * it (the checker) they run one after another with the same results.  The
 * betweenness ranges are fixed by nparts, not by the thread count, and are
 * added in range order, so the sum does not depend on the threads.        */
/* ---------------------------------------------------------------------- */

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Triangles with rows spread over the threads in dynamic chunks. */
int64_t orc_tc_par(int64_t n, const int64_t *rp, const int32_t *ci, int64_t stride)
{
    int64_t t = 0;
    if (stride < 1) stride = 1;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : t)
    for (int64_t u = 0; u < n; u += stride) t += orc_tc_rows(n, rp, ci, u, u + 1, 1);
    return t;
}

/* Queue BFS and the smallest parents from each of ns sources: levels and
 * parents are ns x n, source k in row k. */
int orc_bfs_sources(int64_t n, const int64_t *rp, const int32_t *ci, int64_t ns, const int64_t *sources,
                    int32_t *levels, int64_t *parents)
{
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc)
    for (int64_t k = 0; k < ns; k++) {
        int32_t *lv = levels + k * n;
        int64_t *pa = parents + k * n;
        int r = orc_bfs(n, rp, ci, sources[k], lv, pa);
        if (r == 0) orc_bfs_min_parent(n, rp, ci, sources[k], lv, pa);
        if (r < rc) rc = r;
    }
    return rc;
}

/* Betweenness over ns sources cut into nparts contiguous ranges: each range
 * summed by orc_brandes into part[k * n ...], then the ranges added in
 * order into centrality.  part holds nparts x n doubles. */
int orc_brandes_parts(int64_t n, const int64_t *rp, const int32_t *ci, int64_t ns, const int64_t *sources,
                      int64_t nparts, double *part, double *centrality)
{
    int rc = 0;
    if (nparts < 1) nparts = 1;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc)
    for (int64_t k = 0; k < nparts; k++) {
        const int64_t lo = ns * k / nparts, hi = ns * (k + 1) / nparts;
        int r = orc_brandes(n, rp, ci, hi - lo, sources + lo, part + k * n);
        if (r < rc) rc = r;
    }
    for (int64_t v = 0; v < n; v++) {
        double c = part[v];
        for (int64_t k = 1; k < nparts; k++) c += part[k * n + v];
        centrality[v] = c;
    }
    return rc;
}
