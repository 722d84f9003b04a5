/*
 * CPU oracle for Brandes betweenness centrality on an unweighted CSR graph.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library neither links nor calls it, and it shares no code with the GPU
 * library.
 *
 * What it computes follows the paper's BC specification (Section
 * "Background", the ComputeBC listing), which runs Brandes' algorithm:
 *
 *   BC = 0 once per call.
 *   For each source src of the source set, in the given order:
 *     sigma = 0, delta = 0, sigma[src] = 1.
 *     Forward pass (iterateInBFS): vertices are visited in BFS order from src
 *       and each one sums sigma over its neighbours.
 *     Backward pass (iterateInReverse, v != src): vertices are visited in
 *       reverse BFS order and each one sums (sigma[v]/sigma[w]) * (1+delta[w])
 *       over its neighbours w, then BC[v] += delta[v].
 *
 * Readings of points the listing leaves implicit:
 *   - The neighbour loops run over the BFS DAG: the forward sum takes the
 *     neighbours one level closer to src (the parents), the backward sum the
 *     neighbours one level further (the children).  This is the only reading
 *     that yields Brandes' dependencies, which the paper cites.
 *   - Arithmetic is IEEE double (the listing declares float), the level of a
 *     vertex is an int with -1 for "not reached", as in the generated BFS
 *     kernel the paper prints.
 *   - BC is the raw sum over the given sources: ordered pairs, no 1/2 and no
 *     normalisation; a source repeated k times counts k times.
 *   - A source does not add its own dependency to its BC (v != src).
 *   - Parallel arcs count as distinct paths; self-loops never lie on a
 *     shortest path and have no effect.
 *   - Directed graphs (the *_directed entry points; the CSR lists out-arcs):
 *     the BFS follows arcs forward, sigma sums over parents (arcs into v from
 *     the previous level) and dependencies over children (arcs out of v to the
 *     next level) -- Brandes' algorithm for directed graphs, over the ordered
 *     pairs (s, t) with t reachable from s.
 *
 * Status codes: 0 = ok, 1 = invalid argument, 4 = some sigma is not finite
 * (BC is then written but meaningless).  The *_ext entry points at the end
 * run the same steps in long double for path counts beyond double's range;
 * oracle_sssp is the paper's weighted single-source shortest paths and
 * oracle_pagerank its PageRank.
 *
 * Built with gcc -O2, no fast-math.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_INVALID_ARG = 1, OR_RANGE = 4 };

/* Breadth-first search from s.  dist[v] = hop distance or -1; order[] receives
 * the reached vertices in the order they are dequeued (non-decreasing dist).
 * Returns the number of reached vertices. */
static int32_t bfs_order(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t s,
                         int32_t *dist, int32_t *order) {
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    int32_t head = 0, tail = 0;
    dist[s] = 0;
    order[tail++] = s;
    while (head < tail) {
        int32_t v = order[head++];
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] < 0) {
                dist[w] = dist[v] + 1;
                order[tail++] = w;
            }
        }
    }
    return tail;
}

/* One source: dist, sigma and delta for every vertex.  delta may be NULL
 * (then only the forward pass runs).  bc, when not NULL, receives
 * bc[v] += delta[v] for every reached v != s.  order is scratch of n int32.
 * Returns OR_OK or OR_RANGE.
 *
 * directed = 0: the CSR is symmetric and a vertex's parents are among its
 * neighbours, so sigma is pulled over them.  directed = 1: the CSR lists out-
 * arcs; the BFS follows them, and since a vertex's parents are found through
 * their own out-arcs, each vertex, once its sigma is final (BFS order), adds
 * it to its children (Brandes' formulation).  The reverse pass is the same in
 * both cases: children are reached through out-arcs. */
static int single_source(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t s,
                         int directed, int32_t *dist, double *sigma, double *delta, double *bc,
                         int32_t *order) {
    int32_t reached = bfs_order(n, row_ptr, col_idx, s, dist, order);

    /* sigma = 0 everywhere, sigma[src] = 1. */
    for (int32_t v = 0; v < n; ++v) sigma[v] = 0.0;
    sigma[s] = 1.0;

    int status = OR_OK;
    if (directed) {
        /* Forward pass, BFS order: sigma[v] is final when v is reached in the
         * order; it is added to every child of v. */
        for (int32_t i = 0; i < reached; ++i) {
            int32_t v = order[i];
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t w = col_idx[e];
                if (dist[w] == dist[v] + 1) sigma[w] = sigma[w] + sigma[v];
            }
        }
        for (int32_t i = 1; i < reached; ++i)
            if (!isfinite(sigma[order[i]])) status = OR_RANGE;
    } else {
        /* Forward pass, BFS order: sigma[v] = sum of sigma over parents. */
        for (int32_t i = 1; i < reached; ++i) {
            int32_t v = order[i];
            double acc = 0.0;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t w = col_idx[e];
                if (dist[w] == dist[v] - 1) acc = acc + sigma[w];
            }
            sigma[v] = acc;
            if (!isfinite(acc)) status = OR_RANGE;
        }
    }
    if (delta == NULL) return status;

    /* Backward pass, reverse BFS order, v != src:
     * delta[v] = sum over children w of (sigma[v]/sigma[w]) * (1 + delta[w]). */
    for (int32_t v = 0; v < n; ++v) delta[v] = 0.0;
    for (int32_t i = reached - 1; i >= 1; --i) {
        int32_t v = order[i];
        double acc = 0.0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] == dist[v] + 1) acc = acc + (sigma[v] / sigma[w]) * (1.0 + delta[w]);
        }
        delta[v] = acc;
        if (bc) bc[v] = bc[v] + delta[v];
    }
    return status;
}

static int check_graph_args(int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
    if (n < 0 || (n > 0 && row_ptr == NULL)) return OR_INVALID_ARG;
    if (n > 0 && row_ptr[n] > 0 && col_idx == NULL) return OR_INVALID_ARG;
    return OR_OK;
}

/* dist[n], sigma[n], delta[n] (delta may be NULL) for one source. */
int oracle_single_source(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t s,
                         int32_t *dist, double *sigma, double *delta) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || s < 0 || s >= n || !dist || !sigma)
        return OR_INVALID_ARG;
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int st = single_source(n, row_ptr, col_idx, s, 0, dist, sigma, delta, NULL, order);
    free(order);
    return st;
}

/* As oracle_single_source for a directed graph (row_ptr / col_idx list out-arcs). */
int oracle_single_source_directed(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                  int32_t s, int32_t *dist, double *sigma, double *delta) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || s < 0 || s >= n || !dist || !sigma)
        return OR_INVALID_ARG;
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int st = single_source(n, row_ptr, col_idx, s, 1, dist, sigma, delta, NULL, order);
    free(order);
    return st;
}

/* bc[n] = sum over the k sources of their dependencies.  Sources are split
 * statically over `threads` threads (0 = all available); each thread keeps its
 * own partial BC, and the partials are added in thread order, so the result
 * does not depend on scheduling.  With one thread the sources are processed in
 * the given order. */
static int run_bc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                  const int32_t *sources, int32_t k, int threads, int directed, double *bc) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || k < 0 || !bc ||
        (k > 0 && !sources))
        return OR_INVALID_ARG;
    for (int32_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= n) return OR_INVALID_ARG;
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;
    if (k == 0 || n == 0) return OR_OK;

    int nt = 1;
#ifdef _OPENMP
    nt = threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
#endif
    if (nt > k) nt = k;
    double *partial = (double *)calloc((size_t)nt * (size_t)n, sizeof(double));
    int status = OR_OK;
#pragma omp parallel num_threads(nt) reduction(max : status)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int32_t lo = (int32_t)((int64_t)k * t / nt), hi = (int32_t)((int64_t)k * (t + 1) / nt);
        int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        double *sigma = (double *)malloc((size_t)n * sizeof(double));
        double *delta = (double *)malloc((size_t)n * sizeof(double));
        double *mine = partial + (size_t)t * (size_t)n;
        for (int32_t i = lo; i < hi; ++i) {
            int st = single_source(n, row_ptr, col_idx, sources[i], directed, dist, sigma, delta,
                                   mine, order);
            if (st > status) status = st;
        }
        free(dist);
        free(order);
        free(sigma);
        free(delta);
    }
    for (int t = 0; t < nt; ++t) {
        const double *p = partial + (size_t)t * (size_t)n;
        for (int32_t v = 0; v < n; ++v) bc[v] = bc[v] + p[v];
    }
    free(partial);
    return status;
}

int oracle_bc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *sources,
              int32_t k, int threads, double *bc) {
    return run_bc(n, row_ptr, col_idx, sources, k, threads, 0, bc);
}

/* As oracle_bc for a directed graph (row_ptr / col_idx list out-arcs): ordered
 * pairs (s, t) with t reachable from s along arcs. */
int oracle_bc_directed(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       const int32_t *sources, int32_t k, int threads, double *bc) {
    return run_bc(n, row_ptr, col_idx, sources, k, threads, 1, bc);
}

/* ---- single-source shortest paths ---------------------------------------------
 *
 * The paper's SSSP (Sections "fixedPoint Construct" and "Min/Max
 * Constructs"): dist = infinity everywhere but dist[src] = 0, modified[src] =
 * true; a fixed-point loop runs while some vertex is modified.  Each pass visits
 * the modified vertices v (in id order) and, for each out-arc (v, nbr) of weight
 * w, applies <nbr.dist, nbr.modified_next> = <Min(nbr.dist, v.dist + w), true>
 * (both only when the new distance is smaller); then modified = modified_next
 * and modified_next is cleared.  Distances are updated in place, as in the
 * generated code.  Weights are non-negative integers; distances are 64-bit.
 * dist[v] = -1 where v is unreachable.  Returns the number of passes (>= 1),
 * or -1 for invalid arguments (a negative weight included). */
int64_t oracle_sssp(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                    const int32_t *weight, int32_t s, int64_t *dist) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || s < 0 || s >= n || !dist ||
        (row_ptr[n] > 0 && !weight))
        return -1;
    for (int64_t e = 0; e < row_ptr[n]; ++e)
        if (weight[e] < 0) return -1;
    const int64_t inf = INT64_MAX;
    char *modified = (char *)calloc((size_t)n, 1);
    char *modified_next = (char *)calloc((size_t)n, 1);
    for (int32_t v = 0; v < n; ++v) dist[v] = inf;
    dist[s] = 0;
    modified[s] = 1;
    int64_t passes = 0;
    int finished = 0;
    while (!finished) {
        finished = 1;
        ++passes;
        for (int32_t v = 0; v < n; ++v) {
            if (!modified[v]) continue;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t nbr = col_idx[e];
                int64_t dist_new = dist[v] + weight[e];
                if (dist[nbr] > dist_new) {
                    dist[nbr] = dist_new;
                    modified_next[nbr] = 1;
                    finished = 0;
                }
            }
        }
        char *t = modified;
        modified = modified_next;
        modified_next = t;
        memset(modified_next, 0, (size_t)n);
    }
    for (int32_t v = 0; v < n; ++v)
        if (dist[v] == inf) dist[v] = -1;
    free(modified);
    free(modified_next);
    return passes;
}

/* ---- PageRank -------------------------------------------------------------------
 *
 * The paper's PageRank (the generated loop of Section "Backend Optimizations",
 * OpenACC reduction): every vertex starts at 1/n; an iteration computes, for
 * each v, sum = sum over the arcs u->v of pr[u] / outdeg(u) (pulled over the
 * reversed CSR, in-neighbours in ascending id order), val = (1 - damping)/n +
 * damping * sum, diff += |val - pr[v]|, pr_next[v] = val; then pr = pr_next.
 * Iterations stop once diff <= tol or after max_iter of them.  The listing
 * accumulates the signed difference val - pr[v], which sums to zero whenever no
 * rank leaks (it would stop after one iteration); the L1 norm is taken instead.
 * The CSR lists out-arcs (for an undirected graph, both arcs of an edge).
 * pr[n] receives the result; returns the iterations run (>= 1), or -1 for
 * invalid arguments. */
int64_t oracle_pagerank(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        double damping, double tol, int32_t max_iter, double *pr,
                        double *last_diff) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || !pr || max_iter < 1 ||
        !(damping >= 0.0 && damping <= 1.0) || !(tol >= 0.0))
        return -1;
    if (n == 0) return 1;
    const int64_t nnz = row_ptr[n];
    /* reversed CSR by counting sort: in-neighbours in ascending id order */
    int32_t *in_rp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *in_ci = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    for (int64_t e = 0; e < nnz; ++e) in_rp[col_idx[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) in_rp[v + 1] += in_rp[v];
    int32_t *fill = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) fill[v] = in_rp[v];
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) in_ci[fill[col_idx[e]]++] = u;
    double *next = (double *)malloc((size_t)n * sizeof(double));
    for (int32_t v = 0; v < n; ++v) pr[v] = 1.0 / (double)n;
    int64_t iter = 0;
    double diff = 0.0;
    do {
        diff = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            double sum = 0.0;
            for (int32_t e = in_rp[v]; e < in_rp[v + 1]; ++e) {
                int32_t u = in_ci[e];
                sum = sum + pr[u] / (double)(row_ptr[u + 1] - row_ptr[u]);
            }
            double val = (1.0 - damping) / (double)n + damping * sum;
            diff = diff + fabs(val - pr[v]);
            next[v] = val;
        }
        for (int32_t v = 0; v < n; ++v) pr[v] = next[v];
        ++iter;
    } while (diff > tol && iter < max_iter);
    if (last_diff) *last_diff = diff;
    free(in_rp);
    free(in_ci);
    free(fill);
    free(next);
    return iter;
}

/* ---- extended range --------------------------------------------------------
 *
 * The same steps with sigma and delta held in long double (the x86 80-bit
 * extended format: 64-bit significand, exponents to about +-16382), for graphs
 * whose path counts pass double's range -- deep grids without shortcuts,
 * chains of diamonds.  Extended-range counts are a reading beyond the paper,
 * whose listing declares float: only the number format changes, not the
 * algorithm.  sigma leaves as (m, e) with sigma = m * 2^e, 0.5 <= m < 1
 * (m = 0, e = 0 where sigma = 0); delta and BC fit double. */

static int single_source_ld(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            int32_t s, int32_t *dist, long double *sigma, long double *delta,
                            long double *bc, int32_t *order) {
    int32_t reached = bfs_order(n, row_ptr, col_idx, s, dist, order);
    for (int32_t v = 0; v < n; ++v) sigma[v] = 0.0L;
    sigma[s] = 1.0L;
    int status = OR_OK;
    for (int32_t i = 1; i < reached; ++i) {
        int32_t v = order[i];
        long double acc = 0.0L;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] == dist[v] - 1) acc = acc + sigma[w];
        }
        sigma[v] = acc;
        if (!isfinite(acc)) status = OR_RANGE;
    }
    if (delta == NULL) return status;
    for (int32_t v = 0; v < n; ++v) delta[v] = 0.0L;
    for (int32_t i = reached - 1; i >= 1; --i) {
        int32_t v = order[i];
        long double acc = 0.0L;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] == dist[v] + 1) acc = acc + (sigma[v] / sigma[w]) * (1.0L + delta[w]);
        }
        delta[v] = acc;
        if (bc) bc[v] = bc[v] + delta[v];
    }
    return status;
}

/* Significand bits of long double (64 for the x86 extended format). */
int oracle_ld_digits(void) { return LDBL_MANT_DIG; }

/* dist[n], sigma as (sig_m[n], sig_e[n]), delta[n] (may be NULL) for one source. */
int oracle_single_source_ext(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int32_t s, int32_t *dist, double *sig_m, int32_t *sig_e,
                             double *delta) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || s < 0 || s >= n || !dist || !sig_m ||
        !sig_e)
        return OR_INVALID_ARG;
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    long double *sigma = (long double *)malloc((size_t)n * sizeof(long double));
    long double *dl = delta ? (long double *)malloc((size_t)n * sizeof(long double)) : NULL;
    int st = single_source_ld(n, row_ptr, col_idx, s, dist, sigma, dl, NULL, order);
    for (int32_t v = 0; v < n; ++v) {
        int e = 0;
        sig_m[v] = (double)frexpl(sigma[v], &e);
        sig_e[v] = e;
        if (delta) delta[v] = (double)dl[v];
    }
    free(order);
    free(sigma);
    free(dl);
    return st;
}

/* As oracle_bc, with the counts in long double (partials added in thread
 * order in long double, then rounded to double). */
int oracle_bc_ext(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                  const int32_t *sources, int32_t k, int threads, double *bc) {
    if (check_graph_args(n, row_ptr, col_idx) != OR_OK || k < 0 || !bc ||
        (k > 0 && !sources))
        return OR_INVALID_ARG;
    for (int32_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= n) return OR_INVALID_ARG;
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;
    if (k == 0 || n == 0) return OR_OK;
    int nt = 1;
#ifdef _OPENMP
    nt = threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
#endif
    if (nt > k) nt = k;
    long double *partial = (long double *)calloc((size_t)nt * (size_t)n, sizeof(long double));
    int status = OR_OK;
#pragma omp parallel num_threads(nt) reduction(max : status)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int32_t lo = (int32_t)((int64_t)k * t / nt), hi = (int32_t)((int64_t)k * (t + 1) / nt);
        int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        long double *sigma = (long double *)malloc((size_t)n * sizeof(long double));
        long double *delta = (long double *)malloc((size_t)n * sizeof(long double));
        long double *mine = partial + (size_t)t * (size_t)n;
        for (int32_t i = lo; i < hi; ++i) {
            int st = single_source_ld(n, row_ptr, col_idx, sources[i], dist, sigma, delta, mine,
                                      order);
            if (st > status) status = st;
        }
        free(dist);
        free(order);
        free(sigma);
        free(delta);
    }
    for (int32_t v = 0; v < n; ++v) {
        long double acc = 0.0L;
        for (int t = 0; t < nt; ++t) acc = acc + partial[(size_t)t * (size_t)n + v];
        bc[v] = (double)acc;
    }
    free(partial);
    return status;
}

/* Number of threads oracle_bc uses when asked for all of them. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
