/*
 * bcmi -- Brandes betweenness centrality for unweighted directed graphs on AMD Instinct
 * MI355X (gfx950).  C ABI of libbcmi.so.
 *
 * What is computed (section I of S. Quader, "Study of Betweenness Centrality Algorithms
 * in GPU"): the betweenness of v is the share of pairwise shortest paths passing through
 * v, here the raw sum over ordered pairs s != v != t of sigma_st(v) / sigma_st, where
 * sigma_st counts shortest directed s->t paths and sigma_st(v) those with v as an
 * interior vertex.  Unreachable pairs contribute 0; no normalisation is applied.  The
 * method is Brandes' (section I): per source, a level-synchronous breadth-first sweep
 * records BFS distances and shortest-path counts sigma, then a backward sweep over the
 * levels accumulates the dependencies delta into BC.
 *
 * Precision: distances int32 (-1 = unreachable); sigma exact uint64; a source whose
 * counts exceed 2^64-1 is detected exactly and recounted in double precision; delta and
 * BC are double precision.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (hipMalloc'd or torch CUDA tensors) on the
 *     current HIP device; h_* are host pointers.  The caller owns every array it passes.
 *     The library owns the graph's CSR/CSC arrays and all scratch memory until the handle
 *     is freed.
 *   - `stream` is a hipStream_t (NULL = the null stream).  bc_build_csr, bc_exact,
 *     bc_sampled and bc_batch are stream-ordered: their device work follows what the caller
 *     queued on `stream` before the call, and work queued after it sees their results.
 *     bc_build_csr also waits for its build before returning.  Passing a non-NULL `info`
 *     makes a call wait for its own work on that stream and fill `info` before returning.
 *   - Calls that share a graph handle must be ordered with respect to each other (one
 *     stream, or synchronised): the handle's per-source scratch is reused between calls.
 *   - Return value: BC_OK (0) or a negative error code; bc_last_error() gives a message.
 *     Output parameters are written only on BC_OK.  No C++ exception crosses this ABI.
 *   - Vertex ids are uint32 in [0, n); 1 <= n <= 2^31-1; after de-duplication the edge
 *     count must stay below 2^32.  m = 0 is legal (all BC values are 0).
 */
#ifndef BCMI_BC_H
#define BCMI_BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define BC_API __attribute__((visibility("default")))
#else
#define BC_API
#endif

typedef int32_t bc_status;
#define BC_OK 0
#define BC_PENDING 1     /* bc_serve_poll: request not finished yet */
#define BC_E_INVAL (-1)  /* null / negative / inconsistent argument */
#define BC_E_RANGE (-2)  /* vertex id >= n, n out of range, edge count >= 2^32 */
#define BC_E_NOMEM (-3)  /* device allocation failed, or request larger than a server budget */
#define BC_E_HIP (-4)    /* HIP runtime error (message via bc_last_error) */
#define BC_E_STATE (-5)  /* unknown ticket, destroyed handle, stopped server */

typedef struct bc_graph_s* bc_graph;
typedef struct bc_server_s* bc_server;

/* Launch / strategy knobs.  0 in any field means "choose automatically" (autotuner cache,
 * or built-in defaults when tuning is switched off with BCMI_TUNE=off). */
typedef struct {
    int32_t wg_size;            /* threads per workgroup, multiple of 64 in [64, 1024] */
    int32_t wgs_per_source;     /* workgroups cooperating on one source (1, 2, 4, 8), or on one
                                   64-source batch of the batched kernel (1..64; 0 = automatic:
                                   the grid split over min(batches, compute units / 4) batches,
                                   at most one XCD's share each) */
    int32_t sources_per_launch; /* concurrent sources (per-source state slots) */
    int32_t hub_threshold;      /* out-degree from which a vertex is expanded by a whole
                                   wavefront rather than one thread; < 0 = never */
    int32_t lds_max_n;          /* largest n run by the LDS-resident path; < 0 = never */
    int32_t use_graph;          /* 1 = replay a captured hipGraph, -1 = plain launches */
    int32_t batched;            /* 1 = 64 sources per batch (one per wavefront lane),
                                   -1 = one source per workgroup,
                                   3 = one source per workgroup with each BFS level held in
                                       LDS hash tables (deep graphs: lattices, meshes);
                                       switched off (BC_E_INVAL) until a device fault of its
                                       first run is explained,
                                   2 = an earlier levels-in-LDS kernel, removed: BC_E_INVAL */
    int32_t batch_wg_size;      /* workgroup size of the batched kernel: 256, 512, 1024
                                   (0 = automatic: 512, three per compute unit) */
    int32_t batch_pull;         /* batched kernel, direction of the forward sweep: a level is
                                   built from the unreached vertices' in-edges (pulled) instead
                                   of its entries' out-edges when (in-edges of vertices some
                                   source has not reached) * 16 < (out-edges of the level's
                                   entries) * batch_pull; < 0 = always pushed (0 = automatic: 32) */
    int32_t deterministic;      /* 1 = fixed summation order, for debugging: the one-source-per-
                                   workgroup kernel with state in global memory, each workgroup
                                   taking a static share of the sources in order, each vertex's
                                   successor sum in CSR order, and BC reduced from per-workgroup
                                   partial arrays (grid x n doubles) in workgroup order.  Two calls
                                   with the same inputs and knobs then return the same bits, except
                                   for sources whose counts pass 2^64 (their double-precision counts
                                   are summed in arrival order).  Single-graph calls only; slower.
                                   0 or < 0 = off */
} bc_tuning;

typedef struct {
    uint32_t n_sources;             /* sources processed */
    uint32_t n_sigma_fp64_fallback; /* sources whose path counts overflowed uint64 */
    uint32_t levels_max;            /* deepest BFS (number of levels) over the sources */
    uint32_t path;                  /* 0 = one source per workgroup, state in global memory;
                                       1 = one source per workgroup, state in LDS;
                                       2 = 64-source batches;
                                       3 = (removed) an earlier levels-in-LDS kernel;
                                       4, 5, 6 = bc_paper_strategy 1, 2, 3;
                                       7 = one source per workgroup, levels in LDS tables
                                           (sources handed on counted in batch_handoffs) */
    double kernel_ms;               /* device time of the call (HIP events) */
    double t_submit_ms, t_start_ms, t_done_ms; /* bc_serve_poll only: server clock */
    uint64_t reached;               /* sum over sources of vertices reached (source included) */
    uint64_t examined;              /* sum over sources of out-edges of reached vertices */
    uint64_t dag_edges;             /* sum over sources of shortest-path DAG edges */
    uint64_t batch_entries;         /* path 2: (vertex, level) entries of the batches' lists */
    uint64_t batch_edge_visits;     /* path 2: out-edges of those entries */
    uint64_t batch_scans;           /* path 2: level-collect passes (each reads every vertex's masks) */
    uint64_t batch_handoffs;        /* paths 2, 7: sources handed to the one-source-per-workgroup
                                       kernel with state in global memory (path 2: 32-bit count cap,
                                       list capacity or level cap; path 7: a level wider than the
                                       LDS tables) */
    uint64_t batch_cycles[3];       /* path 2: workgroup clock cycles summed over workgroups, in the
                                       forward sweep, the backward sweep, and state reset */
    uint64_t batch_pull_edges;      /* path 2: in-edges read by pulled forward levels */
    uint64_t batch_pull_levels;     /* path 2: forward levels pulled, summed over batches (each reads
                                       every vertex's masks once) */
    uint64_t batch_pull_skipped;    /* path 2: out-edges of the entries of pulled levels, which the
                                       forward sweep did not read */
    uint64_t batch_pull_pairs;      /* path 2: DAG (edge, source) pairs found by pulled levels */
} bc_info;

/* Build a graph handle from a pair list (section II-D: edge list A[i]=u, B[i]=v).
 * d_src, d_dst: m_in uint32 device arrays.  Self-loops and repeated pairs are dropped.
 * The handle holds CSR (row offsets n+1, successor ids sorted per row) and CSC (the
 * transpose) on the device.  Errors: BC_E_INVAL (null/negative), BC_E_RANGE (id >= n, or
 * more than 2^32-1 pairs), BC_E_NOMEM.  The call waits for the build to finish. */
BC_API bc_status bc_build_csr(int32_t n, int64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                       void* stream, bc_graph* out);

/* n and the de-duplicated edge count. */
BC_API bc_status bc_graph_info(bc_graph g, int32_t* n, int64_t* m);

/* Device pointers of the handle's CSR (row_ptr n+1, col m) and CSC (col_ptr n+1, row m);
 * read-only, valid until bc_graph_free. Any output pointer may be NULL. */
BC_API bc_status bc_graph_arrays(bc_graph g, const uint32_t** d_row_ptr, const uint32_t** d_col,
                          const uint32_t** d_csc_ptr, const uint32_t** d_csc_row);

/* Device pointers of the handle's batching order, the order in which the batched path groups
 * sources (64 per batch).  Vertices are ranked outward from a hub h (the vertex of largest
 * in-degree among those with out-edges, lowest id on ties) along reversed edges: vertices at
 * distance k from h (k <= 64) follow every vertex nearer to h and are ranked by (lowest rank
 * among their successors at distance k-1, floor(log2 out-degree) descending, id); the rest
 * follow by (floor(log2 out-degree) descending, id), vertices without out-edges last.
 * d_order: n vertex ids in rank order; d_rank: n ranks (d_rank[d_order[i]] == i).  Both NULL
 * for a graph without edges.  Read-only, valid until bc_graph_free; either output may be NULL. */
BC_API bc_status bc_graph_order(bc_graph g, const uint32_t** d_order, const uint32_t** d_rank);

/* Release the handle and every device buffer it owns (waits for the device). */
BC_API bc_status bc_graph_free(bc_graph g);

/* Exact BC (section I): every vertex is a source.  d_bc: n doubles, overwritten. */
BC_API bc_status bc_exact(bc_graph g, double* d_bc, const bc_tuning* t, void* stream, bc_info* info);

/* Partial BC over a multiset of k sources: d_bc[v] = sum_i [s_i != v] delta_{s_i}(v), no
 * n/k scaling (the sampled-source approximation cited in section I sums the same terms).
 * d_sources: k uint32 device array, each < n (checked on the device; a bad id makes the
 * call return BC_E_RANGE when `info` is given, and is skipped otherwise).  k = 0 zeroes
 * d_bc. */
BC_API bc_status bc_sampled(bc_graph g, const uint32_t* d_sources, int32_t k, double* d_bc,
                     const bc_tuning* t, void* stream, bc_info* info);

/* BC as bc_sampled (k >= 0) or bc_exact (k < 0 with d_sources NULL), also reporting which
 * sources needed the double-precision recount.  Section II-D keeps path counts in 4-byte
 * integers and is silent on overflow; here a source overflows when one of its shortest-path
 * counts exceeds 2^64-1, which is detected exactly (carry out of the 64-bit addition).
 * d_overflowed: n bytes (device), overwritten: 1 at the id of every source of the call whose
 * counts overflowed, 0 everywhere else.  A source listed several times is flagged once.  Other
 * arguments, errors and stream semantics as bc_sampled. */
BC_API bc_status bc_sampled_flags(bc_graph g, const uint32_t* d_sources, int32_t k, double* d_bc,
                                  uint8_t* d_overflowed, const bc_tuning* t, void* stream, bc_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): bc_sampled's result from a call that allocates
 * nothing.  It runs the one-source-per-workgroup kernel with its per-source state in one fixed
 * 32 MiB array of device memory that the library holds on each GPU it runs on until the process
 * ends (one state slot takes 24 n + 4 bytes, so n must be at most 1,398,079: larger graphs get
 * BC_E_RANGE; fewer slots fit as n grows, which bounds the concurrency, not the result).  Every
 * call on a GPU reuses that GPU's array: calls that overlap on one GPU (two streams, two
 * threads) race and must be ordered by the caller.  The graph must be built (bc_build_csr
 * allocates) before.  Arguments as bc_sampled; `t` may set wg_size and hub_threshold (the other
 * fields are ignored).  Stream-ordered, no host synchronisation; bad source ids are skipped.
 * Errors: BC_E_INVAL, BC_E_RANGE (n too large), BC_E_HIP. */
BC_API bc_status bc_sampled_noalloc(bc_graph g, const uint32_t* d_sources, int32_t k, double* d_bc,
                                    const bc_tuning* t, void* stream);

/* One source, for inspection (section I: the BFS distances d(s,.) and shortest-path counts
 * sigma(s,.) exactly as the forward sweep leaves them, and the dependencies delta_s(.) of the
 * backward sweep).  d_dist (int32 n),
 * d_sigma_u64 (uint64 n; exact counts, all 0 when overflowed), d_sigma_f64 (double n;
 * counts as doubles, the double-precision recount when overflowed), d_delta (double n;
 * delta_s(v), delta_s(s) = reached-1).  Any of the four may be NULL.  *h_overflowed is set
 * to 1 when the counts exceeded uint64.  Synchronous. */
BC_API bc_status bc_sssp(bc_graph g, uint32_t s, int32_t* d_dist, uint64_t* d_sigma_u64,
                  double* d_sigma_f64, double* d_delta, int32_t* h_overflowed, void* stream);

/* Exact BC of many independent graphs in one persistent launch.  d_bcs[i] (n_i doubles,
 * overwritten) receives graph i's result.  infos (nullable) has num_graphs entries. */
BC_API bc_status bc_batch(const bc_graph* gs, int32_t num_graphs, double* const* d_bcs,
                   const bc_tuning* t, void* stream, bc_info* infos);

/* Autotune the launch knobs for this graph (times candidate configurations on a sample of
 * sources; cached per device and graph class): workgroup size, hub threshold, state home,
 * sources per launch, and for the batched kernel its workgroup size, workgroups per batch and
 * pull threshold.  Section III-E's observation, that the best block size depends on the graph
 * and is not simply the largest, is why these are searched rather than fixed.  Writes the
 * chosen knobs to *out.  Synchronous.  Errors: BC_E_INVAL (null handle or out), BC_E_HIP. */
BC_API bc_status bc_tune(bc_graph g, bc_tuning* out);

/* Approximate BC from pivot sources (the sampling approximation cited in section I): k
 * pivots drawn uniformly with replacement (SplitMix64 from `seed`), sampled BC scaled by n/k,
 * an unbiased estimate of every BC(v).  k = ceil(ln(2n/delta) / (2 eps^2)), so that with
 * probability >= 1 - delta every |estimate(v) - BC(v)| <= eps * n * (n - 2) (Hoeffding and a
 * union bound over the n vertices); when k >= n the exact BC is computed instead (k = n).
 * eps in (0, 1], delta in (0, 1).  d_bc: n doubles, overwritten.  k_out (nullable): k.
 * h_pivots (nullable, host, capacity pivots_cap >= k): the pivots used (0..n-1 when exact).
 * info (nullable) as for bc_sampled.  Errors: BC_E_INVAL, BC_E_NOMEM, BC_E_HIP.  Returns after
 * the work is done. */
BC_API bc_status bc_approx(bc_graph g, double eps, double delta, uint64_t seed, double* d_bc, int32_t* k_out,
                           uint32_t* h_pivots, int32_t pivots_cap, void* stream, bc_info* info);

/* Adaptive sampling for one vertex v: pivots (same generator) are taken in rounds of 64 until
 * the sampled dependencies S = sum delta_s(v) reach c * n or max_samples pivots were used;
 * the estimate n * S / k is written to *h_est (host), k to *k_out (nullable), the pivots to
 * h_pivots (nullable, capacity pivots_cap >= max_samples).  Errors: BC_E_INVAL (c <= 0,
 * max_samples <= 0, null estimate), BC_E_RANGE (v >= n), BC_E_NOMEM, BC_E_HIP. */
BC_API bc_status bc_approx_vertex(bc_graph g, uint32_t v, double c, uint64_t seed, int32_t max_samples,
                                  double* h_est, int32_t* k_out, uint32_t* h_pivots, int32_t pivots_cap,
                                  void* stream);

/* The three GPU strategies compared in the paper (section I, section III), rebuilt as baselines
 * for rerunning that comparison on its own workload (BA digraphs); not the fast path:
 *   strategy 1: one workgroup per source, vertex-parallel levels (every vertex tested each
 *               level, a vertex's successors walked by one thread);
 *   strategy 2: one workgroup per source, edge-parallel levels over the edge list;
 *   strategy 3: one source at a time over the whole grid, one launch per level, the host
 *               reading an "another level?" flag after each forward launch.
 * wg_size: threads per workgroup, multiple of 64 in [64, 1024] (the paper's block-size study).
 * d_sources: k device source ids (multiset, raw sum; NULL allowed when k = 0); k < 0 = all n
 * vertices (exact BC).
 * d_bc: n doubles, overwritten with the same BC as bc_exact / bc_sampled (sigma is held in
 * double precision here, exact below 2^53).  info (nullable): n_sources, levels_max,
 * kernel_ms, path = 3 + strategy.  Errors: BC_E_INVAL (strategy, wg_size, null output),
 * BC_E_RANGE (a source id >= n), BC_E_NOMEM, BC_E_HIP.  Returns after the work is done. */
BC_API bc_status bc_paper_strategy(bc_graph g, int32_t strategy, int32_t wg_size, const uint32_t* d_sources,
                                   int32_t k, double* d_bc, void* stream, bc_info* info);

/* ---- serving ------------------------------------------------------------------------
 * A server owns a device stream and a host thread.  Requests are admitted while the sum
 * of their device footprints (graph CSR+CSC, per-source state slots, output) fits
 * `hbm_budget_bytes`; the rest wait in arrival order.  Admitted requests are cut into
 * source chunks and executed together (continuous batching): requests that arrive while
 * others run join the next launch.  All bc_serve_* calls are thread-safe. */
BC_API bc_status bc_serve_create(size_t hbm_budget_bytes, int32_t max_slots, bc_server* out);

/* Submit BC of graph g over h_sources (host array of k ids; NULL = every vertex, exact)
 * into d_bc (n doubles, overwritten when the request completes).  The graph handle and
 * d_bc must stay valid until the ticket completes.  Never blocks on device work.
 * BC_E_NOMEM if the request alone exceeds the server budget. */
BC_API bc_status bc_serve_submit(bc_server s, bc_graph g, const uint32_t* h_sources, int32_t k,
                          double* d_bc, uint64_t* ticket);

/* BC_OK and *info filled when the ticket is complete, BC_PENDING otherwise. */
BC_API bc_status bc_serve_poll(bc_server s, uint64_t ticket, bc_info* info);

/* Stop the server: queued requests are cancelled, running ones are finished first. */
BC_API bc_status bc_serve_destroy(bc_server s);

/* Measurement utility, not part of the method: the HBM bandwidth that plain streaming reaches
 * on the current device.  STREAM-style copy (b = a) and triad (a = b + q c) over arrays of
 * `bytes` each (choose far more than the 256 MB MALL), timed with HIP events, median of `reps`
 * runs after one warm-up run.  Writes GB/s counting 2 (copy) or 3 (triad) array sizes moved per
 * run into the non-NULL host outputs.  Allocates and frees three device arrays; synchronous.
 * Errors: BC_E_INVAL (bytes < 16, reps < 1), BC_E_NOMEM, BC_E_HIP. */
BC_API bc_status bc_stream_probe(size_t bytes, int32_t reps, double* h_copy_gbs, double* h_triad_gbs);

/* Thread-local message of the last error on this thread ("" if none). */
BC_API const char* bc_last_error(void);

/* Library version string. */
BC_API const char* bc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BCMI_BC_H */
