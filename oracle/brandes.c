/*
 * CPU oracle for Brandes betweenness centrality on unweighted directed graphs.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the device path is checked against.  Nothing in the product
 * library links it; only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, headers or tables with the device
 * path.
 *
 * What it computes (section I of the paper): BC(v) is the share of all
 * pairwise shortest paths that pass through v, summed over ordered pairs:
 *
 *     BC(v) = sum over s != v != t of sigma_st(v) / sigma_st
 *
 * with sigma_st the number of shortest s->t paths and sigma_st(v) those of
 * them that visit v as an interior vertex; pairs with t unreachable add 0.
 * The raw (unnormalised) sum is returned.
 *
 * How (section I, Brandes' O(nm)-time, O(n+m)-space method): for each source
 * s, one breadth-first search gives the BFS distance d(s,.) and the number of
 * shortest paths sigma(s,.); then the dependency of s on v,
 *
 *     delta_s(v) = sum over successors w of v with d(s,w) = d(s,v)+1 of
 *                  (sigma(s,v) / sigma(s,w)) * (1 + delta_s(w)),
 *
 * is accumulated in reverse BFS order, and BC(v) += delta_s(v) for v != s.
 *
 * Precision: distances int32 (-1 = unreachable); sigma exact uint64.  If any
 * addition into sigma carries past 2^64-1 the source is flagged as overflowed
 * and its search is repeated with sigma in double precision.  delta and BC are
 * double precision.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------------------
 * Simple-graph adjacency (section II-D, adjacency-list format): the input is a list of
 * ordered pairs; self-loops and repeated pairs are dropped, since the method is defined on
 * simple digraphs (a repeated edge would double-count paths).  Each vertex's successor list
 * is returned in increasing id order.  Returns the number of kept edges, or -1 on an id
 * outside [0, n).
 * ------------------------------------------------------------------------------------- */
static int cmp_pair(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

int64_t oracle_simple_adjacency(int32_t n, int64_t m_in, const uint32_t* src, const uint32_t* dst,
                                uint32_t* row_ptr, uint32_t* col) {
    uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m_in > 0 ? m_in : 1));
    if (!pairs) return -2;
    int64_t kept = 0;
    for (int64_t i = 0; i < m_in; ++i) {
        if (src[i] >= (uint32_t)n || dst[i] >= (uint32_t)n) { free(pairs); return -1; }
        if (src[i] == dst[i]) continue;
        pairs[kept++] = ((uint64_t)src[i] << 32) | dst[i];
    }
    qsort(pairs, (size_t)kept, sizeof(uint64_t), cmp_pair);
    int64_t m = 0;
    for (int32_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    for (int64_t i = 0; i < kept; ++i) {
        if (i > 0 && pairs[i] == pairs[i - 1]) continue;
        uint32_t u = (uint32_t)(pairs[i] >> 32);
        col[m++] = (uint32_t)(pairs[i] & 0xffffffffu);
        row_ptr[u + 1] += 1;
    }
    for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    free(pairs);
    return m;
}

/* Per-source work counters: reached vertices |R_s| (s included), examined edges |E_s|
 * (out-edges of reached vertices), shortest-path DAG edges |D_s|, number of BFS levels. */
typedef struct {
    int64_t reached, examined, dag_edges, levels;
} oracle_stats;

/* ---------------------------------------------------------------------------------------
 * One source, steps as in section I's description of Brandes' method.
 *   dist[n]      BFS distance from s, -1 if unreachable
 *   sigma[n]     exact shortest-path counts (valid iff *overflow == 0)
 *   sigma_f[n]   shortest-path counts as doubles (exact conversion of sigma when no
 *                overflow; the double-precision re-count when overflowed)
 *   delta[n]     dependency of s on each vertex (delta[s] is filled too, never added to BC)
 *   order[n]     scratch: BFS visit order
 * ------------------------------------------------------------------------------------- */
static void bfs_count(int32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t s,
                      int32_t* dist, uint64_t* sigma, double* sigma_f, int use_double,
                      uint32_t* order, int64_t* n_order, int* overflow, oracle_stats* st) {
    for (int32_t v = 0; v < n; ++v) { dist[v] = -1; sigma[v] = 0; sigma_f[v] = 0.0; }
    dist[s] = 0;
    sigma[s] = 1;
    sigma_f[s] = 1.0;
    int64_t head = 0, tail = 0;
    order[tail++] = s;
    int64_t examined = 0, dag = 0;
    int32_t deepest = 0;
    *overflow = 0;
    while (head < tail) {
        uint32_t v = order[head++];
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t w = col[e];
            ++examined;
            if (dist[w] < 0) {                    /* first visit: w is one level deeper */
                dist[w] = dist[v] + 1;
                if (dist[w] > deepest) deepest = dist[w];
                order[tail++] = w;
            }
            if (dist[w] == dist[v] + 1) {         /* (v,w) lies on a shortest path */
                ++dag;
                if (use_double) {
                    sigma_f[w] += sigma_f[v];
                } else {
                    uint64_t sum;
                    if (__builtin_add_overflow(sigma[w], sigma[v], &sum)) *overflow = 1;
                    sigma[w] = sum;
                }
            }
        }
    }
    if (!use_double)
        for (int64_t i = 0; i < tail; ++i) sigma_f[order[i]] = (double)sigma[order[i]];
    *n_order = tail;
    st->reached = tail;
    st->examined = examined;
    st->dag_edges = dag;
    st->levels = (int64_t)deepest + 1;
}

int oracle_brandes_source(int32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t s,
                          int32_t* dist, uint64_t* sigma, double* sigma_f, double* delta,
                          uint32_t* order, int32_t* overflow_out, oracle_stats* st) {
    if (s >= (uint32_t)n) return -1;
    int64_t count = 0;
    int overflow = 0;
    bfs_count(n, row_ptr, col, s, dist, sigma, sigma_f, 0, order, &count, &overflow, st);
    if (overflow)   /* exact counts do not fit in 64 bits: count again in double precision */
        bfs_count(n, row_ptr, col, s, dist, sigma, sigma_f, 1, order, &count, &overflow, st),
        overflow = 1;
    for (int32_t v = 0; v < n; ++v) delta[v] = 0.0;
    /* dependencies, deepest vertices first (reverse BFS order) */
    for (int64_t i = count - 1; i >= 0; --i) {
        uint32_t v = order[i];
        double acc = 0.0;
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t w = col[e];
            if (dist[w] == dist[v] + 1)
                acc += (sigma_f[v] / sigma_f[w]) * (1.0 + delta[w]);
        }
        delta[v] = acc;
    }
    *overflow_out = overflow;
    return 0;
}

/* ---------------------------------------------------------------------------------------
 * BC over a multiset of sources: bc[v] = sum over i of [sources[i] != v] * delta_{s_i}(v).
 * With sources = every vertex once this is exact BC; otherwise the raw partial sum (no
 * n/k scaling).  Sources are split statically over `threads` OpenMP threads, each keeps
 * its own BC array, and the arrays are added in thread order, so a fixed thread count
 * gives a fixed result.
 *   overflowed[k]  (nullable) 1 where that source's counts exceeded 64 bits
 *   stats[4*k]     (nullable) reached, examined, dag_edges, levels per source
 * ------------------------------------------------------------------------------------- */
int oracle_bc(int32_t n, const uint32_t* row_ptr, const uint32_t* col, const uint32_t* sources,
              int64_t k, double* bc, uint8_t* overflowed, int64_t* stats, int threads) {
    for (int64_t i = 0; i < k; ++i)
        if (sources[i] >= (uint32_t)n) return -1;
    if (threads < 1) threads = 1;
    double* partial = (double*)calloc((size_t)threads * (size_t)n, sizeof(double));
    if (!partial) return -2;
    int failed = 0;
#pragma omp parallel num_threads(threads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        uint64_t* sigma = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        double* sigma_f = (double*)malloc(sizeof(double) * (size_t)n);
        double* delta = (double*)malloc(sizeof(double) * (size_t)n);
        uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
        double* mine = partial + (size_t)tid * (size_t)n;
        if (!dist || !sigma || !sigma_f || !delta || !order) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < k; ++i) {
                uint32_t s = sources[i];
                int32_t ovf = 0;
                oracle_stats st;
                oracle_brandes_source(n, row_ptr, col, s, dist, sigma, sigma_f, delta, order, &ovf, &st);
                for (int32_t v = 0; v < n; ++v)
                    if ((uint32_t)v != s) mine[v] += delta[v];
                if (overflowed) overflowed[i] = (uint8_t)ovf;
                if (stats) {
                    stats[4 * i + 0] = st.reached;
                    stats[4 * i + 1] = st.examined;
                    stats[4 * i + 2] = st.dag_edges;
                    stats[4 * i + 3] = st.levels;
                }
            }
        }
        free(dist); free(sigma); free(sigma_f); free(delta); free(order);
    }
    for (int32_t v = 0; v < n; ++v) {
        double acc = 0.0;
        for (int t = 0; t < threads; ++t) acc += partial[(size_t)t * (size_t)n + v];
        bc[v] = acc;
    }
    free(partial);
    return failed ? -2 : 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
