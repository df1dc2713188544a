// C ABI of libbcmi.so: argument checks, error mapping, graph handles, and the
// single-graph entry points.  Batch, tuning and serving live in their own files.
#include "bc_internal.h"

#include <algorithm>
#include <atomic>
#include <vector>

#include <cstdio>

namespace bcmi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

void graph_scratch_free(Graph& g);
void batch_forget_graph(const Graph* g);

Graph::Graph() {
    static std::atomic<uint64_t> next{1};
    uid = next.fetch_add(1);
}

Graph::~Graph() {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    // a cached batch plan that lists this graph would replay its freed arrays
    batch_forget_graph(this);
    graph_scratch_free(*this);
    strat_pool_delete(strat);
    if (row_ptr) (void)hipFree(row_ptr);
    if (col) (void)hipFree(col);
    if (csc_ptr) (void)hipFree(csc_ptr);
    if (csc_row) (void)hipFree(csc_row);
    if (perm) (void)hipFree(perm);
    if (iperm) (void)hipFree(iperm);
    if (prow) (void)hipFree(prow);
    if (rank) (void)hipFree(rank);
    if (order) (void)hipFree(order);
    if (pcol) (void)hipFree(pcol);
    if (stats) (void)hipFree(stats);
    (void)hipSetDevice(prev);
}

const DevInfo& dev_info(int device) {
    static std::mutex mu;
    static std::vector<DevInfo*> cache;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= device) cache.resize(device + 1, nullptr);
    if (!cache[device]) {
        DevInfo* d = new DevInfo();
        hipDeviceProp_t prop;
        BC_HIP_TRY(hipGetDeviceProperties(&prop, device));
        d->cus = prop.multiProcessorCount;
        d->lds_per_block = (int)prop.sharedMemPerBlock;
        d->max_threads = prop.maxThreadsPerBlock;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess && v > 0)
            d->lds_per_cu = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
            v > d->lds_per_block)
            d->lds_per_block = v;
        d->name = prop.gcnArchName;
        cache[device] = d;
    }
    return *cache[device];
}

// Runs `body`, converting exceptions to a status code and message.
template <class F>
static bc_status guarded(F&& body) {
    try {
        clear_error();
        body();
        return BC_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return BC_E_NOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return BC_E_HIP;
    } catch (...) {
        set_error("unknown failure");
        return BC_E_HIP;
    }
}

static Graph* as_graph(bc_graph g) {
    BC_REQUIRE(g != nullptr, BC_E_INVAL, "null graph handle");
    return reinterpret_cast<Graph*>(g);
}

// Event pair that times a stretch of one stream.
struct StreamTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit StreamTimer(hipStream_t s, bool on) : st(s) {
        if (!on) return;
        BC_HIP_TRY(hipEventCreate(&a));
        BC_HIP_TRY(hipEventCreate(&b));
        BC_HIP_TRY(hipEventRecord(a, st));
    }
    double stop_ms() {
        if (!a) return 0.0;
        BC_HIP_TRY(hipEventRecord(b, st));
        BC_HIP_TRY(hipEventSynchronize(b));
        float ms = 0.f;
        BC_HIP_TRY(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~StreamTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

void graph_discard_batched_state(Graph& g);

static void fill_info(Graph& g, hipStream_t st, int path, double ms, uint32_t expected, bc_info* info) {
    CallStats cs;
    read_stats(g, st, &cs);
    if (cs.aborted) {
        graph_discard_batched_state(g);
        throw Error{BC_E_HIP, "batched kernel: a team of workgroups stopped waiting at a level barrier"};
    }
    BC_REQUIRE(cs.bad_source == 0, BC_E_RANGE, "a source id is >= n");
    BC_REQUIRE(cs.n_done == expected, BC_E_HIP, "not every source completed");
    bc_info out{};
    out.n_sources = cs.n_done;
    out.n_sigma_fp64_fallback = cs.n_overflow;
    out.levels_max = cs.levels_max;
    out.path = (uint32_t)path;
    out.kernel_ms = ms;
    out.reached = cs.reached;
    out.examined = cs.examined;
    out.dag_edges = cs.dag_edges;
    out.batch_entries = cs.entries;
    out.batch_edge_visits = cs.edge_visits;
    out.batch_scans = cs.scans;
    out.batch_handoffs = cs.handoffs;
    for (int i = 0; i < 3; ++i) out.batch_cycles[i] = cs.cycles[i];
    out.batch_pull_edges = cs.pull_edges;
    out.batch_pull_levels = cs.pull_levels;
    out.batch_pull_skipped = cs.pull_skip;
    out.batch_pull_pairs = cs.pull_pairs;
    *info = out;
}

}  // namespace bcmi

using namespace bcmi;

extern "C" {

const char* bc_last_error(void) { return g_last_error.c_str(); }

const char* bc_version(void) { return "bcmi 0.1 (gfx950)"; }

bc_status bc_build_csr(int32_t n, int64_t m_in, const uint32_t* d_src, const uint32_t* d_dst, void* stream,
                       bc_graph* out) {
    return guarded([&] {
        BC_REQUIRE(out != nullptr, BC_E_INVAL, "null output handle");
        BC_REQUIRE(n >= 1, BC_E_RANGE, "n must be >= 1");
        BC_REQUIRE(m_in >= 0, BC_E_INVAL, "m_in must be >= 0");
        Graph* g = new Graph();
        try {
            BC_HIP_TRY(hipGetDevice(&g->device));
            build_csr_device(n, m_in, d_src, d_dst, (hipStream_t)stream, *g);
        } catch (...) {
            delete g;
            throw;
        }
        *out = reinterpret_cast<bc_graph>(g);
    });
}

bc_status bc_graph_info(bc_graph gh, int32_t* n, int64_t* m) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        if (n) *n = g->n;
        if (m) *m = g->m;
    });
}

bc_status bc_graph_arrays(bc_graph gh, const uint32_t** row_ptr, const uint32_t** col, const uint32_t** csc_ptr,
                          const uint32_t** csc_row) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        if (row_ptr) *row_ptr = g->row_ptr;
        if (col) *col = g->col;
        if (csc_ptr) *csc_ptr = g->csc_ptr;
        if (csc_row) *csc_row = g->csc_row;
    });
}

bc_status bc_graph_order(bc_graph gh, const uint32_t** order, const uint32_t** rank) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        if (order) *order = g->order;
        if (rank) *rank = g->rank;
    });
}

bc_status bc_graph_free(bc_graph gh) {
    return guarded([&] { delete as_graph(gh); });
}

bc_status bc_sampled(bc_graph gh, const uint32_t* d_sources, int32_t k, double* d_bc, const bc_tuning* t,
                     void* stream, bc_info* info) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        BC_REQUIRE(k >= 0, BC_E_INVAL, "k must be >= 0");
        BC_REQUIRE(k == 0 || d_sources != nullptr, BC_E_INVAL, "null source array");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const Knobs kn = resolve_knobs(*g, t);
        RunArgs ra{};
        ra.g = g;
        ra.sources = d_sources;
        ra.num_items = (uint32_t)k;
        ra.bc = d_bc;
        StreamTimer tm(st, info != nullptr);
        const int path = run_sources(ra, kn, st, *g);
        if (info) {
            const double ms = tm.stop_ms();
            fill_info(*g, st, path, ms, (uint32_t)k, info);
        }
    });
}

bc_status bc_sampled_flags(bc_graph gh, const uint32_t* d_sources, int32_t k, double* d_bc, uint8_t* d_overflowed,
                           const bc_tuning* t, void* stream, bc_info* info) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        BC_REQUIRE(d_overflowed != nullptr, BC_E_INVAL, "null overflow-flag array");
        BC_REQUIRE(k >= 0 || d_sources == nullptr, BC_E_INVAL, "k < 0 (every vertex) takes no source array");
        BC_REQUIRE(k <= 0 || d_sources != nullptr, BC_E_INVAL, "null source array");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const Knobs kn = resolve_knobs(*g, t);
        RunArgs ra{};
        ra.g = g;
        ra.sources = k < 0 ? nullptr : d_sources;
        ra.num_items = k < 0 ? (uint32_t)g->n : (uint32_t)k;
        ra.bc = d_bc;
        ra.ovf_flags = d_overflowed;
        StreamTimer tm(st, info != nullptr);
        const int path = run_sources(ra, kn, st, *g);
        if (info) {
            const double ms = tm.stop_ms();
            fill_info(*g, st, path, ms, ra.num_items, info);
        }
    });
}

bc_status bc_exact(bc_graph gh, double* d_bc, const bc_tuning* t, void* stream, bc_info* info) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const Knobs kn = resolve_knobs(*g, t);
        RunArgs ra{};
        ra.g = g;
        ra.sources = nullptr;
        ra.num_items = (uint32_t)g->n;
        ra.bc = d_bc;
        StreamTimer tm(st, info != nullptr);
        const int path = run_sources(ra, kn, st, *g);
        if (info) {
            const double ms = tm.stop_ms();
            fill_info(*g, st, path, ms, (uint32_t)g->n, info);
        }
    });
}

bc_status bc_sssp(bc_graph gh, uint32_t s, int32_t* d_dist, uint64_t* d_sigma_u64, double* d_sigma_f64,
                  double* d_delta, int32_t* h_overflowed, void* stream) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(s < (uint32_t)g->n, BC_E_RANGE, "source id >= n");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        Knobs kn = resolve_knobs(*g, nullptr);
        uint32_t* d_src = nullptr;
        double* d_bc = nullptr;
        BC_HIP_TRY(hipMallocAsync((void**)&d_src, sizeof(uint32_t), st));
        BC_HIP_TRY(hipMallocAsync((void**)&d_bc, sizeof(double) * g->n, st));
        BC_HIP_TRY(hipMemcpyAsync(d_src, &s, sizeof(uint32_t), hipMemcpyHostToDevice, st));
        RunArgs ra{};
        ra.g = g;
        ra.sources = d_src;
        ra.num_items = 1;
        ra.bc = d_bc;
        ra.ex_dist = d_dist;
        ra.ex_sigma = d_sigma_u64;
        ra.ex_sigma_f = d_sigma_f64;
        ra.ex_delta = d_delta;
        run_sources(ra, kn, st, *g);
        CallStats cs;
        read_stats(*g, st, &cs);
        (void)hipFreeAsync(d_src, st);
        (void)hipFreeAsync(d_bc, st);
        BC_HIP_TRY(hipStreamSynchronize(st));
        BC_REQUIRE(cs.n_done == 1, BC_E_HIP, "search did not complete");
        if (h_overflowed) *h_overflowed = cs.n_overflow ? 1 : 0;
    });
}

}  // extern "C"

namespace bcmi {
void run_batch(const bc_graph* gs, int num, double* const* bcs, const bc_tuning* t, hipStream_t st, bc_info* infos,
               double* kernel_ms);
Knobs tune_graph(Graph& g);
}  // namespace bcmi

extern "C" {

bc_status bc_batch(const bc_graph* gs, int32_t num_graphs, double* const* d_bcs, const bc_tuning* t, void* stream,
                   bc_info* infos) {
    return guarded([&] {
        BC_REQUIRE(num_graphs >= 0, BC_E_INVAL, "num_graphs must be >= 0");
        if (num_graphs == 0) return;
        BC_REQUIRE(gs && d_bcs, BC_E_INVAL, "null graph or output list");
        int dev = 0;
        BC_HIP_TRY(hipGetDevice(&dev));
        for (int i = 0; i < num_graphs; ++i) {
            Graph* g = as_graph(gs[i]);
            BC_REQUIRE(d_bcs[i] != nullptr, BC_E_INVAL, "null output array");
            BC_REQUIRE(g->device == dev, BC_E_INVAL, "graph lives on another device");
        }
        run_batch(gs, num_graphs, d_bcs, t, (hipStream_t)stream, infos, nullptr);
    });
}

bc_status bc_approx(bc_graph gh, double eps, double delta, uint64_t seed, double* d_bc, int32_t* k_out,
                    uint32_t* h_pivots, int32_t pivots_cap, void* stream, bc_info* info) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        const uint32_t n = (uint32_t)g->n;
        const uint32_t k = hoeffding_pivots(n, eps, delta);
        BC_REQUIRE(h_pivots == nullptr || pivots_cap >= (int32_t)k, BC_E_INVAL, "pivot buffer too small");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const Knobs kn = resolve_knobs(*g, nullptr);
        RunArgs ra{};
        ra.g = g;
        ra.bc = d_bc;
        std::vector<uint32_t> piv;
        uint32_t* d_piv = nullptr;
        if (k < n) {   // pivots, scaled by n/k
            piv.resize(k);
            draw_pivots(seed, n, k, piv.data());
            BC_HIP_TRY(hipMalloc((void**)&d_piv, sizeof(uint32_t) * std::max<uint32_t>(k, 1)));
            ra.sources = d_piv;
            ra.num_items = k;
        } else {       // the bound asks for n pivots or more: exact BC
            ra.sources = nullptr;
            ra.num_items = n;
        }
        try {
            if (d_piv) BC_HIP_TRY(hipMemcpyAsync(d_piv, piv.data(), sizeof(uint32_t) * k, hipMemcpyHostToDevice, st));
            StreamTimer tm(st, info != nullptr);
            const int path = run_sources(ra, kn, st, *g);
            if (k < n) scale_bc(d_bc, n, (double)n / (double)k, st);
            if (info) {
                const double ms = tm.stop_ms();
                fill_info(*g, st, path, ms, ra.num_items, info);
            }
            BC_HIP_TRY(hipStreamSynchronize(st));
        } catch (...) {
            if (d_piv) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(d_piv);
            }
            throw;
        }
        if (d_piv) (void)hipFree(d_piv);
        if (k_out) *k_out = (int32_t)k;
        if (h_pivots) {
            if (k < n) std::copy(piv.begin(), piv.end(), h_pivots);
            else for (uint32_t i = 0; i < n; ++i) h_pivots[i] = i;
        }
    });
}

bc_status bc_approx_vertex(bc_graph gh, uint32_t v, double c, uint64_t seed, int32_t max_samples, double* h_est,
                           int32_t* k_out, uint32_t* h_pivots, int32_t pivots_cap, void* stream) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(h_est != nullptr, BC_E_INVAL, "null estimate pointer");
        BC_REQUIRE(c > 0.0, BC_E_INVAL, "c must be > 0");
        BC_REQUIRE(max_samples > 0, BC_E_INVAL, "max_samples must be > 0");
        const uint32_t n = (uint32_t)g->n;
        BC_REQUIRE(v < n, BC_E_RANGE, "vertex id >= n");
        BC_REQUIRE(h_pivots == nullptr || pivots_cap >= max_samples, BC_E_INVAL, "pivot buffer too small");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const Knobs kn = resolve_knobs(*g, nullptr);
        constexpr uint32_t kRound = 64;   // pivots per round: one batch of the batched kernel
        std::vector<uint32_t> piv((size_t)max_samples);
        draw_pivots(seed, n, (uint32_t)max_samples, piv.data());
        uint32_t* d_piv = nullptr;
        double* d_part = nullptr;
        double* d_tmp = nullptr;
        double sum = 0.0;
        uint32_t taken = 0;
        try {
            BC_HIP_TRY(hipMalloc((void**)&d_piv, sizeof(uint32_t) * piv.size()));
            BC_HIP_TRY(hipMalloc((void**)&d_part, sizeof(double) * std::max<uint32_t>(n, 1)));
            BC_HIP_TRY(hipMalloc((void**)&d_tmp, sizeof(double)));
            BC_HIP_TRY(hipMemcpyAsync(d_piv, piv.data(), sizeof(uint32_t) * piv.size(), hipMemcpyHostToDevice, st));
            while (taken < (uint32_t)max_samples && sum < c * (double)n) {
                const uint32_t r = std::min<uint32_t>(kRound, (uint32_t)max_samples - taken);
                RunArgs ra{};
                ra.g = g;
                ra.bc = d_part;
                ra.sources = d_piv + taken;
                ra.num_items = r;
                run_sources(ra, kn, st, *g);
                sum += read_bc_entry(d_part, v, d_tmp, st);   // the round's sum of delta_s(v)
                taken += r;
            }
        } catch (...) {
            (void)hipStreamSynchronize(st);
            for (void* q : {(void*)d_piv, (void*)d_part, (void*)d_tmp})
                if (q) (void)hipFree(q);
            throw;
        }
        for (void* q : {(void*)d_piv, (void*)d_part, (void*)d_tmp})
            if (q) (void)hipFree(q);
        *h_est = taken ? (double)n * sum / (double)taken : 0.0;
        if (k_out) *k_out = (int32_t)taken;
        if (h_pivots) std::copy(piv.begin(), piv.begin() + taken, h_pivots);
    });
}

bc_status bc_paper_strategy(bc_graph gh, int32_t strategy, int32_t wg_size, const uint32_t* d_sources, int32_t k,
                            double* d_bc, void* stream, bc_info* info) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        BC_REQUIRE(k <= 0 || d_sources != nullptr, BC_E_INVAL, "null source array");
        std::lock_guard<std::mutex> lk(g->mu);
        const hipStream_t st = (hipStream_t)stream;
        const bool all = k < 0;
        const uint32_t items = all ? (uint32_t)g->n : (uint32_t)k;
        if (!all && k > 0) {   // the kernels trust their source ids
            std::vector<uint32_t> h(k);
            BC_HIP_TRY(hipMemcpyAsync(h.data(), d_sources, sizeof(uint32_t) * k, hipMemcpyDeviceToHost, st));
            BC_HIP_TRY(hipStreamSynchronize(st));
            for (uint32_t x : h) BC_REQUIRE(x < (uint32_t)g->n, BC_E_RANGE, "a source id is >= n");
        }
        StreamTimer tm(st, info != nullptr);
        uint32_t levels = 0;
        run_strategy(g->strat, *g, strategy, wg_size, all ? nullptr : d_sources, items, d_bc, st, &levels);
        if (info) {
            bc_info out{};
            out.kernel_ms = tm.stop_ms();
            out.n_sources = items;
            out.levels_max = levels;
            out.path = (uint32_t)(3 + strategy);
            *info = out;
        }
    });
}

bc_status bc_sampled_noalloc(bc_graph gh, const uint32_t* d_sources, int32_t k, double* d_bc, const bc_tuning* t,
                             void* stream) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(d_bc != nullptr, BC_E_INVAL, "null output array");
        BC_REQUIRE(k >= 0, BC_E_INVAL, "k must be >= 0");
        BC_REQUIRE(k == 0 || d_sources != nullptr, BC_E_INVAL, "null source array");
        const Knobs kn = resolve_knobs(*g, t);
        run_sampled_noalloc(*g, d_sources, (uint32_t)k, d_bc, kn, (hipStream_t)stream);
    });
}

bc_status bc_stream_probe(size_t bytes, int32_t reps, double* h_copy_gbs, double* h_triad_gbs) {
    return guarded([&] { stream_probe(bytes, reps, h_copy_gbs, h_triad_gbs); });
}

bc_status bc_tune(bc_graph gh, bc_tuning* out) {
    return guarded([&] {
        Graph* g = as_graph(gh);
        BC_REQUIRE(out != nullptr, BC_E_INVAL, "null output");
        std::lock_guard<std::mutex> lk(g->mu);
        const Knobs k = tune_graph(*g);
        bc_tuning r{};
        r.wg_size = k.wg_size;
        r.wgs_per_source = k.team;
        r.sources_per_launch = k.teams;
        r.hub_threshold = k.hub;
        r.lds_max_n = k.lds_max_n;
        r.use_graph = k.use_graph ? 1 : -1;
        r.batched = k.batched;
        r.batch_wg_size = k.batch_wg;
        r.batch_pull = k.batch_pull > 0 ? k.batch_pull : -1;
        *out = r;
    });
}

}  // extern "C"
