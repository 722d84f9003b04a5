/*
 * Seeded synthetic graph inputs for Brandes betweenness centrality.
 *
 * These generators build the unweighted, undirected inputs that stand in for
 * the paper's graph suite (Section "Experimental Evaluation", the input-graph
 * table): a skewed R-MAT graph with quadrant probabilities
 * a=0.57, b=0.19, c=0.19, d=0.05, a road-like 2D grid, and a uniform random
 * graph.  They hold none of the centrality arithmetic: both the CPU oracle and
 * the GPU library consume the CSR arrays produced here.
 *
 * Every random draw is a pure function of (seed, stream, counter), so the
 * output does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* splitmix64 finaliser (Steele, Lea, Flood 2014) used as a counter-based
 * generator: draw i of stream s under seed k is mix(mix(k ^ s*phi) + i*phi). */
static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t ctr_draw(uint64_t key, uint64_t i) {
    return mix64(key + i * 0x9E3779B97F4A7C15ULL);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(seed ^ (stream * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL));
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Exported for the Python side, so that every draw comes from one definition. */
uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t i) {
    return ctr_draw(stream_key(seed, stream), i);
}

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of m edges picks one of four
 * quadrants per bit of the vertex id, with probabilities a, b, c, 1-a-b-c.
 * No noise is added.  Endpoints go to src[i], dst[i]. */
void gg_rmat_edges(int scale, int64_t m, double a, double b, double c, uint64_t seed,
                   int32_t *src, int32_t *dst) {
    const uint64_t key = stream_key(seed, 1);
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint32_t u = 0, v = 0;
        for (int j = 0; j < scale; ++j) {
            double r = u01(ctr_draw(key, (uint64_t)i * (uint64_t)scale + (uint64_t)j));
            uint32_t ubit = 0, vbit = 0;
            if (r < a) {
            } else if (r < ab) {
                vbit = 1;
            } else if (r < abc) {
                ubit = 1;
            } else {
                ubit = 1;
                vbit = 1;
            }
            u = (u << 1) | ubit;
            v = (v << 1) | vbit;
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
}

/* Uniform random permutation of 0..n-1 (Fisher-Yates, draws from stream 9). */
void gg_permutation(int32_t n, uint64_t seed, int32_t *perm) {
    const uint64_t key = stream_key(seed, 9);
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        uint64_t r = ctr_draw(key, (uint64_t)i);
        int32_t j = (int32_t)(r % (uint64_t)(i + 1));
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

/* Apply a relabelling in place: x -> perm[x]. */
void gg_relabel(int64_t m, const int32_t *perm, int32_t *src, int32_t *dst) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        src[i] = perm[src[i]];
        dst[i] = perm[dst[i]];
    }
}

/* G(n, m): m edges with endpoints uniform over 0..n-1 (stream 4). */
void gg_uniform_edges(int32_t n, int64_t m, uint64_t seed, int32_t *src, int32_t *dst) {
    const uint64_t key = stream_key(seed, 4);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        src[i] = (int32_t)(u01(ctr_draw(key, 2 * (uint64_t)i)) * (double)n);
        dst[i] = (int32_t)(u01(ctr_draw(key, 2 * (uint64_t)i + 1)) * (double)n);
    }
}

/* rows x cols 4-neighbour grid, vertex id r*cols+c.  Edge e (horizontal edges
 * first, row-major, then vertical) is kept when its draw from stream 2 is
 * >= remove_frac.  Then `n_shortcuts` edges with uniform endpoints (stream 3)
 * are appended.  Returns the number of edges written (capacity must be at
 * least 2*rows*cols + n_shortcuts). */
int64_t gg_grid_edges(int32_t rows, int32_t cols, double remove_frac, int64_t n_shortcuts,
                      uint64_t seed, int32_t *src, int32_t *dst) {
    const uint64_t kkeep = stream_key(seed, 2), kshort = stream_key(seed, 3);
    const int64_t n = (int64_t)rows * cols;
    int64_t e = 0, w = 0;
    for (int32_t r = 0; r < rows; ++r)
        for (int32_t c = 0; c + 1 < cols; ++c, ++e)
            if (u01(ctr_draw(kkeep, (uint64_t)e)) >= remove_frac) {
                src[w] = r * cols + c;
                dst[w] = r * cols + c + 1;
                ++w;
            }
    for (int32_t r = 0; r + 1 < rows; ++r)
        for (int32_t c = 0; c < cols; ++c, ++e)
            if (u01(ctr_draw(kkeep, (uint64_t)e)) >= remove_frac) {
                src[w] = r * cols + c;
                dst[w] = (r + 1) * cols + c;
                ++w;
            }
    for (int64_t i = 0; i < n_shortcuts; ++i) {
        src[w] = (int32_t)(u01(ctr_draw(kshort, 2 * (uint64_t)i)) * (double)n);
        dst[w] = (int32_t)(u01(ctr_draw(kshort, 2 * (uint64_t)i + 1)) * (double)n);
        ++w;
    }
    return w;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Edge list -> CSR.  With `symmetrize`, every edge (u,v) yields arcs u->v and
 * v->u.  With `drop_loops`, self-loops are removed.  With `dedup`, repeated
 * arcs collapse to one.  Each adjacency list ends up sorted ascending.
 * row_ptr has n+1 entries; col_idx must hold (symmetrize ? 2m : m) entries.
 * Returns the final arc count, or -1 when it does not fit in int32. */
int64_t gg_csr_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          int symmetrize, int drop_loops, int dedup, int32_t *row_ptr,
                          int32_t *col_idx) {
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        if (drop_loops && src[i] == dst[i]) continue;
        off[src[i] + 1]++;
        if (symmetrize) off[dst[i] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    memcpy(cur, off, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        if (drop_loops && src[i] == dst[i]) continue;
        col_idx[cur[src[i]]++] = dst[i];
        if (symmetrize) col_idx[cur[dst[i]]++] = src[i];
    }
    free(cur);
    int64_t *deg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t v = 0; v < n; ++v) {
        int32_t *a = col_idx + off[v];
        int64_t d = off[v + 1] - off[v];
        qsort(a, (size_t)d, sizeof(int32_t), cmp_i32);
        if (dedup && d > 1) {
            int64_t k = 1;
            for (int64_t j = 1; j < d; ++j)
                if (a[j] != a[k - 1]) a[k++] = a[j];
            d = k;
        }
        deg[v] = d;
    }
    int64_t w = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t s = off[v];
        if (w != s) memmove(col_idx + w, col_idx + s, (size_t)deg[v] * sizeof(int32_t));
        off[v] = w;
        w += deg[v];
    }
    off[n] = w;
    int64_t total = w;
    if (total > INT32_MAX) total = -1;
    else
        for (int32_t v = 0; v <= n; ++v) row_ptr[v] = (int32_t)off[v];
    free(deg);
    free(off);
    return total;
}

/* First k entries of a seeded Fisher-Yates shuffle of 0..count-1 (stream 7):
 * a uniform sample without replacement. */
void gg_sample_without_replacement(int64_t count, int64_t k, uint64_t seed, int64_t *out) {
    const uint64_t key = stream_key(seed, 7);
    int64_t *idx = (int64_t *)malloc((size_t)count * sizeof(int64_t));
    for (int64_t i = 0; i < count; ++i) idx[i] = i;
    for (int64_t i = 0; i < k; ++i) {
        uint64_t r = ctr_draw(key, (uint64_t)i);
        int64_t j = i + (int64_t)(r % (uint64_t)(count - i));
        int64_t t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
        out[i] = idx[i];
    }
    free(idx);
}

/* Arc weights in [lo, hi] (stream 14), for the CSR's arcs in order.  With
 * symmetric != 0 the weight of arc u->v is drawn from the unordered pair
 * {u, v} (index min*n + max), so both arcs of an undirected edge agree;
 * otherwise from the arc (u*n + v). */
void gg_edge_weights(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, uint64_t seed,
                     int32_t lo, int32_t hi, int symmetric, int32_t *w) {
    const uint64_t key = stream_key(seed, 14);
    const uint64_t span = (uint64_t)(hi - lo + 1);
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col_idx[e];
            uint64_t a = (uint64_t)u, b = (uint64_t)v;
            if (symmetric && b < a) {
                a = (uint64_t)v;
                b = (uint64_t)u;
            }
            w[e] = lo + (int32_t)(ctr_draw(key, a * (uint64_t)n + b) % span);
        }
    }
}
