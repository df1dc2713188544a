// Launch knobs: built-in defaults, the autotuner and its cache, explicit caller overrides.
//
// The tuner times candidate configurations (state home, workgroup size, hub threshold, sources
// per launch; for the batched kernel its workgroup size, workgroups per batch and pull threshold;
// batched vs one source per workgroup) on an evenly strided sample of the graph's sources
// and keeps the fastest per graph class: (device, floor(log2 n), round(log2(m/n))).  Results
// live in memory for the process and, when BCMI_TUNE_CACHE names a file, in that JSON file.
// BCMI_TUNE=off makes every call use the built-in defaults.
#include "bc_internal.h"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <sstream>

namespace bcmi {

bool tuning_enabled() {
    const char* e = std::getenv("BCMI_TUNE");
    return !(e && std::string(e) == "off");
}

Knobs default_knobs(const Graph& g) {
    Knobs k;
    k.lds_max_n = 4096;
    // deep graphs (lattice-like) run one source per workgroup through thousands of small
    // levels, and graphs of the LDS-resident path through wide ones: larger workgroups take
    // a level in fewer chunks (batch of 4,096 R-MAT graphs of scale 6..12: 924 -> 698 ms)
    const bool lds = g.n <= k.lds_max_n;
    k.wg_size = g.deep || lds ? 512 : 256;
    k.team = 0;     // batched path: workgroups per batch chosen from the batch count
    k.teams = 0;
    k.hub = lds ? 128 : 64;
    k.use_graph = true;
    k.batched = 0;
    k.batch_wg = 512;
    k.batch_pull = 32;
    return k;
}

namespace {

std::mutex g_cache_mu;
std::map<std::string, Knobs> g_cache;
bool g_cache_loaded = false;

std::string class_key(const Graph& g) {
    const int ln = (int)std::floor(std::log2((double)std::max(g.n, 1)));
    const int ld = (int)std::lround(std::log2(std::max(1.0, (double)g.m / std::max(g.n, 1))));
    std::ostringstream o;
    o << dev_info(g.device).name << "/n" << ln << "/d" << ld;
    return o.str();
}

const char* cache_path() { return std::getenv("BCMI_TUNE_CACHE"); }

void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* p = cache_path();
    if (!p) return;
    FILE* f = std::fopen(p, "r");
    if (!f) return;
    char key[256];
    Knobs k;
    int ug = 0;
    // one entry per line: key wg hub lds_max_n batched batch_wg teams use_graph team batch_pull
    while (std::fscanf(f, "%255s %d %d %d %d %d %d %d %d %d", key, &k.wg_size, &k.hub, &k.lds_max_n, &k.batched,
                       &k.batch_wg, &k.teams, &ug, &k.team, &k.batch_pull) == 10) {
        k.use_graph = ug != 0;
        g_cache[key] = k;
    }
    std::fclose(f);
}

void save_cache_locked() {
    const char* p = cache_path();
    if (!p) return;
    FILE* f = std::fopen(p, "w");
    if (!f) return;
    for (const auto& kv : g_cache) {
        const Knobs& k = kv.second;
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d\n", kv.first.c_str(), k.wg_size, k.hub, k.lds_max_n,
                     k.batched, k.batch_wg, k.teams, k.use_graph ? 1 : 0, k.team, k.batch_pull);
    }
    std::fclose(f);
}

__global__ void k_strided_sources(uint32_t* out, uint32_t k, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
        out[i] = (uint32_t)(((uint64_t)i * n) / k);
}

}  // namespace

Knobs resolve_knobs(Graph& g, const bc_tuning* t) {
    Knobs k = default_knobs(g);
    if (tuning_enabled()) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_cache_locked();
        auto it = g_cache.find(class_key(g));
        if (it != g_cache.end()) k = it->second;
    }
    if (!t) return k;
    if (t->wg_size) {
        BC_REQUIRE(t->wg_size >= 64 && t->wg_size <= 1024 && t->wg_size % 64 == 0, BC_E_INVAL,
                   "wg_size must be a multiple of 64 in [64, 1024]");
        k.wg_size = t->wg_size;
    }
    if (t->wgs_per_source) {
        BC_REQUIRE(t->wgs_per_source >= 1 && t->wgs_per_source <= 64, BC_E_INVAL, "wgs_per_source must be in [1, 64]");
        k.team = t->wgs_per_source;
    }
    if (t->sources_per_launch) {
        BC_REQUIRE(t->sources_per_launch > 0, BC_E_INVAL, "sources_per_launch must be > 0");
        k.teams = t->sources_per_launch;
    }
    if (t->hub_threshold) k.hub = t->hub_threshold;
    if (t->lds_max_n) k.lds_max_n = t->lds_max_n;
    if (t->use_graph) k.use_graph = t->use_graph > 0;
    if (t->batched) {
        BC_REQUIRE(t->batched >= -1 && t->batched <= 3, BC_E_INVAL, "batched must be -1, 0, 1, 2 or 3");
        k.batched = t->batched;
    }
    if (t->batch_pull) k.batch_pull = t->batch_pull;
    if (t->deterministic) k.deterministic = t->deterministic > 0;
    if (t->batch_wg_size) {
        BC_REQUIRE(t->batch_wg_size == 256 || t->batch_wg_size == 512 || t->batch_wg_size == 1024, BC_E_INVAL,
                   "batch_wg_size must be 256, 512 or 1024");
        k.batch_wg = t->batch_wg_size;
    }
    return k;
}

// Times the candidates on a sample of sources and caches the fastest for the graph's class.
Knobs tune_graph(Graph& g) {
    const Knobs base = default_knobs(g);
    std::vector<Knobs> cands;
    const bool small = lds_fits(base, (uint32_t)g.n, g.device);
    const int cus = dev_info(g.device).cus;
    if (small) {
        // workgroup size, hub threshold, and sources per launch (the persistent grid: every
        // resident workgroup, or one per compute unit)
        for (int wg : {64, 128, 256, 512})
            for (int hub : {64, 128})
                for (int teams : {0, cus}) {
                    if (teams && wg < 256) continue;
                    Knobs k = base;
                    k.wg_size = wg;
                    k.hub = hub;
                    k.teams = teams;
                    k.batched = -1;
                    cands.push_back(k);
                }
    } else {
        // batched: workgroup size, workgroups per batch (0 = from the batch count), and the
        // forward's pull threshold
        for (int bwg : {512, 1024})
            for (int team : {0, 2, 8}) {
                Knobs k = base;
                k.batched = 1;
                k.batch_wg = bwg;
                k.team = team;
                cands.push_back(k);
            }
        for (int pull : {16, 64}) {
            Knobs k = base;
            k.batched = 1;
            k.batch_pull = pull;
            cands.push_back(k);
        }
        for (int wg : {256, 512})
            for (int hub : {32, 128}) {
                Knobs k = base;
                k.batched = -1;
                k.lds_max_n = -1;
                k.wg_size = wg;
                k.hub = hub;
                cands.push_back(k);
            }
    }
    const uint32_t sample = (uint32_t)std::min<int64_t>(g.n, g.n >= (1 << 18) ? 512 : 2048);
    hipStream_t st;
    BC_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    uint32_t* d_src = nullptr;
    double* d_bc = nullptr;
    hipEvent_t e0, e1;
    Knobs best = base;
    try {
        BC_HIP_TRY(hipMalloc((void**)&d_src, sizeof(uint32_t) * std::max<uint32_t>(sample, 1)));
        BC_HIP_TRY(hipMalloc((void**)&d_bc, sizeof(double) * g.n));
        BC_HIP_TRY(hipEventCreate(&e0));
        BC_HIP_TRY(hipEventCreate(&e1));
        hipLaunchKernelGGL(k_strided_sources, dim3(std::max(1u, (sample + 255) / 256)), dim3(256), 0, st, d_src, sample,
                           (uint32_t)g.n);
        BC_HIP_TRY(hipGetLastError());
        float best_ms = 1e30f;
        for (const Knobs& k : cands) {
            RunArgs ra{};
            ra.g = &g;
            ra.sources = d_src;
            ra.num_items = sample;
            ra.bc = d_bc;
            run_sources(ra, k, st, g);   // warm-up (allocates the state pools)
            BC_HIP_TRY(hipEventRecord(e0, st));
            run_sources(ra, k, st, g);
            BC_HIP_TRY(hipEventRecord(e1, st));
            BC_HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            BC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = k;
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (d_src) (void)hipFree(d_src);
        if (d_bc) (void)hipFree(d_bc);
        (void)hipStreamDestroy(st);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_src);
    (void)hipFree(d_bc);
    (void)hipStreamDestroy(st);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    load_cache_locked();
    g_cache[class_key(g)] = best;
    save_cache_locked();
    return best;
}

}  // namespace bcmi
