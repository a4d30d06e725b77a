/*
 * Seeded synthetic inputs: R-MAT edge draws and seeded sampling.
 *
 * This file is shared by the oracle and the device path as an INPUT source
 * only.  It holds none of the method's arithmetic: it draws raw (u, v) pairs
 * (self-loops and duplicates included, not symmetrised) and picks seeded
 * subsets.  Building the adjacency matrix from these pairs is done
 * separately on each side.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) used as a
 * counter-based generator: the i-th output of a stream whose state starts
 * at `key` is mix(key + (i + 1) * GAMMA), so any draw can be computed
 * independently of the others and generation parallelises without changing
 * a single bit.
 *
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each edge descends
 * `scale` levels of the adjacency matrix; at each level a uniform r picks
 * the quadrant (0,0) if r < a, (0,1) if r < a+b, (1,0) if r < a+b+c, else
 * (1,1).  The first level decides the most significant bit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t gg_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* First output of a SplitMix64 stream seeded with x. */
uint64_t gg_splitmix64(uint64_t x) { return gg_mix(x + GG_GAMMA); }

/* i-th output (i >= 0) of the stream whose state starts at key. */
static inline uint64_t gg_nth(uint64_t key, uint64_t i)
{
    return gg_mix(key + (i + 1) * GG_GAMMA);
}

static inline double gg_u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Stream key for a (seed, stream-tag) pair. */
static inline uint64_t gg_key(uint64_t seed, uint64_t tag)
{
    return gg_mix(gg_mix(seed + GG_GAMMA) ^ (tag * 0xd1b54a32d192ed03ULL + 1));
}

/*
 * m raw R-MAT draws for a 2^scale vertex graph.  Draw e, level l uses the
 * (e * 64 + l)-th output of stream (seed, tag 0).  src/dst: int32[m].
 */
void gg_rmat_edges(int scale, int64_t m, uint64_t seed, double a, double b,
                   double c, int32_t *src, int32_t *dst)
{
    const uint64_t key = gg_key(seed, 0);
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; l++) {
            const double r = gg_u01(gg_nth(key, (uint64_t)e * 64u + (uint64_t)l));
            const uint32_t bit = 1u << (scale - 1 - l);
            if (r < a) {
            } else if (r < ab) {
                v |= bit;
            } else if (r < abc) {
                u |= bit;
            } else {
                u |= bit;
                v |= bit;
            }
        }
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
    }
}

/* flag[x] = 1 for every vertex that has at least one draw with u != v. */
void gg_touched(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                uint8_t *flag)
{
    memset(flag, 0, (size_t)n);
    for (int64_t e = 0; e < m; e++) {
        if (src[e] != dst[e]) {
            flag[src[e]] = 1;
            flag[dst[e]] = 1;
        }
    }
}

/*
 * k distinct positions drawn without replacement from [0, ncand) by a
 * partial Fisher-Yates shuffle driven by stream (seed, tag).  Returns -1 if
 * k > ncand or memory is short.
 */
int gg_sample(int64_t ncand, int64_t k, uint64_t seed, uint64_t tag,
              int64_t *out)
{
    if (k > ncand || k < 0) return -1;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncand > 0 ? ncand : 1));
    if (!idx) return -1;
    for (int64_t i = 0; i < ncand; i++) idx[i] = i;
    const uint64_t key = gg_key(seed, tag);
    for (int64_t i = 0; i < k; i++) {
        const uint64_t span = (uint64_t)(ncand - i);
        const uint64_t r = gg_nth(key, (uint64_t)i);
        const uint64_t j = (uint64_t)i + (uint64_t)(((unsigned __int128)r * span) >> 64);
        const int64_t t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
        out[i] = idx[i];
    }
    free(idx);
    return 0;
}

/* count uniforms in [0,1) from stream (seed, tag), outputs i0 .. i0+count-1. */
void gg_uniforms(uint64_t seed, uint64_t tag, int64_t i0, int64_t count, double *out)
{
    const uint64_t key = gg_key(seed, tag);
    for (int64_t i = 0; i < count; i++) out[i] = gg_u01(gg_nth(key, (uint64_t)(i0 + i)));
}

/* Symmetric integer edge weights in [1, wmax] for an adjacency in CSR form:
 * entry (u, v) gets 1 + (x mod wmax) where x is output number
 * min(u,v) * 2^32 + max(u,v) of stream (seed, tag), so w(u,v) = w(v,u). */
void gg_edge_weights(int64_t n, const int64_t *rp, const int32_t *ci, uint64_t seed, uint64_t tag,
                     int64_t wmax, double *out)
{
    const uint64_t key = gg_key(seed, tag);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++)
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            const uint64_t v = (uint64_t)ci[p];
            const uint64_t a = (uint64_t)u < v ? (uint64_t)u : v, b = (uint64_t)u < v ? v : (uint64_t)u;
            out[p] = (double)(1 + gg_nth(key, (a << 32) | b) % (uint64_t)wmax);
        }
}
