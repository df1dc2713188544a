// The three GPU strategies the paper compares (section I, section III), rebuilt on gfx950 as
// selectable baselines, so its comparison can be rerun on its own workload (BA digraphs):
//
//   1. vertex-parallel, one workgroup per source: at level d every vertex is tested for
//      dist == d, and a frontier vertex's successors are walked by one thread (the adjacency-
//      list design; load-imbalanced on hubs);
//   2. edge-parallel, one workgroup per source: at level d every edge (u, w) of the edge list
//      is tested for dist[u] == d (neighbourhood-level parallelism);
//   3. edge-parallel over the whole grid for one source at a time, one launch per level, the
//      host reading a "another level?" flag after each forward launch.  The flag is kept per
//      workgroup in LDS and written to global memory once by each workgroup that set it (the
//      paper's code optimisation).
//
// Each strategy computes the same quantities as the main kernels (Brandes' method, successor
// form of the dependency recurrence): dist, sigma, delta per source, and BC[v] += delta[v] for
// v != s.  Differences from the paper's versions, all deliberate:
//   * no predecessor array: the backward sweep tests dist[w] == dist[v] + 1 on successors;
//   * sigma in double precision (exact below 2^53, which the paper's workloads never reach);
//     the paper used 32-bit integers;
//   * state allocated once per call, not per level.
// These kernels are baselines, not the fast path: every level scans all n vertices or all m
// edges.
#include "bc_internal.h"

#include <algorithm>
#include <vector>

namespace bcmi {

namespace {

struct StratArgs {
    const uint32_t* row_ptr;
    const uint32_t* col;
    const uint32_t* coo_src;   // edge e runs coo_src[e] -> col[e]
    uint32_t n, m;
    const uint32_t* sources;   // nullable: item i is source i
    uint32_t items;
    double* bc;
    int32_t* dist;             // [slots][n]
    double* sig;               // [slots][n]
    double* del;               // [slots][n]
    uint32_t* head;            // work counter
    uint32_t* levels_max;
};

__global__ void k_coo_src(const uint32_t* __restrict__ row_ptr, uint32_t n, uint32_t* __restrict__ src) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) src[e] = v;
}

// relaxation of edge u -> w from level d (u on level d): claim, then count
__device__ __forceinline__ bool relax(int32_t* dist, double* sig, uint32_t w, double su, int d) {
    int dw = dist[w];
    bool claimed = false;
    if (dw < 0) {
        const int old = atomicCAS(&dist[w], -1, d + 1);
        claimed = old < 0;
        dw = claimed ? d + 1 : old;
    }
    if (dw == d + 1) atomicAdd(&sig[w], su);
    return claimed;
}

// strategies 1 and 2: a persistent grid, one source per workgroup at a time
template <bool EDGE>
__global__ void k_strategy_block(StratArgs a) {
    __shared__ uint32_t item, more;
    const unsigned tid = threadIdx.x, nt = blockDim.x;
    int32_t* dist = a.dist + (size_t)blockIdx.x * a.n;
    double* sig = a.sig + (size_t)blockIdx.x * a.n;
    double* del = a.del + (size_t)blockIdx.x * a.n;
    for (;;) {
        if (tid == 0) item = atomicAdd(a.head, 1u);
        __syncthreads();
        const uint32_t it = item;
        __syncthreads();
        if (it >= a.items) break;
        const uint32_t s = a.sources ? a.sources[it] : it;   // ids checked by the host
        for (uint32_t v = tid; v < a.n; v += nt) {
            dist[v] = v == s ? 0 : -1;
            sig[v] = v == s ? 1.0 : 0.0;
            del[v] = 0.0;
        }
        __syncthreads();
        int d = 0;
        for (;;) {   // forward: level d -> d + 1
            if (tid == 0) more = 0;
            __syncthreads();
            bool any = false;
            if (EDGE) {
                for (uint32_t e = tid; e < a.m; e += nt) {
                    const uint32_t u = a.coo_src[e];
                    if (dist[u] == d) any |= relax(dist, sig, a.col[e], sig[u], d);
                }
            } else {
                for (uint32_t v = tid; v < a.n; v += nt) {
                    if (dist[v] != d) continue;
                    const double sv = sig[v];
                    for (uint32_t e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e) any |= relax(dist, sig, a.col[e], sv, d);
                }
            }
            if (any) more = 1u;
            __syncthreads();
            const bool go = more != 0u;
            __syncthreads();
            if (!go) break;
            ++d;
        }
        // levels 0..d are populated; level d has no successors on a further level
        for (int dd = d - 1; dd >= 0; --dd) {
            if (EDGE) {   // every DAG edge adds its share into its tail (atomics, as the edge list needs)
                for (uint32_t e = tid; e < a.m; e += nt) {
                    const uint32_t u = a.coo_src[e];
                    if (dist[u] != dd) continue;
                    const uint32_t w = a.col[e];
                    if (dist[w] == dd + 1) atomicAdd(&del[u], sig[u] / sig[w] * (1.0 + del[w]));
                }
            } else {      // each level-dd vertex sums over its own successors
                for (uint32_t v = tid; v < a.n; v += nt) {
                    if (dist[v] != dd) continue;
                    double acc = 0.0;
                    for (uint32_t e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e) {
                        const uint32_t w = a.col[e];
                        if (dist[w] == dd + 1) acc += (1.0 + del[w]) / sig[w];
                    }
                    del[v] = sig[v] * acc;
                }
            }
            __syncthreads();
        }
        for (uint32_t v = tid; v < a.n; v += nt)
            if (v != s && del[v] != 0.0) unsafeAtomicAdd(&a.bc[v], del[v]);
        if (tid == 0) atomicMax(a.levels_max, (uint32_t)(d + 1));
        __syncthreads();
    }
}

// strategy 3: one source at a time over the whole grid
__global__ void k_strat_init(int32_t* dist, double* sig, double* del, uint32_t n, uint32_t s) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        dist[v] = v == s ? 0 : -1;
        sig[v] = v == s ? 1.0 : 0.0;
        del[v] = 0.0;
    }
}

__global__ void k_strat_forward(StratArgs a, int d, uint32_t* flag) {
    __shared__ uint32_t more;   // "another level?" kept in LDS, one global write per workgroup
    if (threadIdx.x == 0) more = 0;
    __syncthreads();
    bool any = false;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < a.m; e += gridDim.x * blockDim.x) {
        const uint32_t u = a.coo_src[e];
        if (a.dist[u] == d) any |= relax(a.dist, a.sig, a.col[e], a.sig[u], d);
    }
    if (any) more = 1u;
    __syncthreads();
    if (threadIdx.x == 0 && more) *flag = 1u;
}

__global__ void k_strat_backward(StratArgs a, int d) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < a.m; e += gridDim.x * blockDim.x) {
        const uint32_t u = a.coo_src[e];
        if (a.dist[u] != d) continue;
        const uint32_t w = a.col[e];
        if (a.dist[w] == d + 1) atomicAdd(&a.del[u], a.sig[u] / a.sig[w] * (1.0 + a.del[w]));
    }
}

__global__ void k_strat_accumulate(const double* del, double* bc, uint32_t n, uint32_t s) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (v != s) bc[v] += del[v];
}

__global__ void k_strat_zero(double* bc, uint32_t n, uint32_t* words, uint32_t nwords) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) bc[v] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x < nwords) words[threadIdx.x] = 0u;
}

}  // namespace

// Device scratch of the strategy baselines (grown on demand, kept with the graph).
struct StratPool {
    uint32_t* coo_src = nullptr;
    uint32_t m = 0;
    int32_t* dist = nullptr;
    double* sig = nullptr;
    double* del = nullptr;
    size_t slot_elems = 0;      // n * slots
    uint32_t* words = nullptr;  // [0] head, [1] levels_max, [2] flag
    uint32_t* h_flag = nullptr; // pinned
};

void strat_pool_delete(StratPool* p) {
    if (!p) return;
    for (void* q : {(void*)p->coo_src, (void*)p->dist, (void*)p->sig, (void*)p->del, (void*)p->words})
        if (q) (void)hipFree(q);
    if (p->h_flag) (void)hipHostFree(p->h_flag);
    delete p;
}

void run_strategy(StratPool*& pool, const Graph& g, int strategy, int wg, const uint32_t* d_sources, uint32_t k,
                  double* d_bc, hipStream_t st, uint32_t* levels_max) {
    BC_REQUIRE(strategy >= 1 && strategy <= 3, BC_E_INVAL, "strategy must be 1, 2 or 3");
    BC_REQUIRE(wg >= 64 && wg <= 1024 && wg % 64 == 0, BC_E_INVAL, "wg_size must be a multiple of 64 in [64, 1024]");
    if (!pool) pool = new StratPool();
    StratPool& p = *pool;
    const uint32_t n = (uint32_t)g.n, m = g.m;
    if (!p.words) {
        BC_HIP_TRY(hipMalloc((void**)&p.words, 4 * sizeof(uint32_t)));
        BC_HIP_TRY(hipHostMalloc((void**)&p.h_flag, sizeof(uint32_t), hipHostMallocDefault));
    }
    if (m > 0 && (!p.coo_src || p.m < m)) {
        BC_HIP_TRY(hipStreamSynchronize(st));
        if (p.coo_src) (void)hipFree(p.coo_src);
        p.coo_src = nullptr;
        BC_HIP_TRY(hipMalloc((void**)&p.coo_src, (size_t)m * sizeof(uint32_t)));
        p.m = m;
    }
    if (m > 0) {
        hipLaunchKernelGGL(k_coo_src, dim3(std::max(1u, std::min((n + 255) / 256, 4096u))), dim3(256), 0, st,
                           g.row_ptr, n, p.coo_src);
        BC_HIP_TRY(hipGetLastError());
    }
    const DevInfo& di = dev_info(g.device);
    // concurrent sources: one state slot per resident workgroup (strategies 1, 2), one slot (3)
    long slots = 1;
    const void* fn = strategy == 1 ? (const void*)k_strategy_block<false> : (const void*)k_strategy_block<true>;
    if (strategy != 3) {
        int per_cu = 0;
        BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, 0));
        BC_REQUIRE(per_cu >= 1, BC_E_HIP, "strategy kernel does not fit on a compute unit");
        slots = std::min<long>((long)per_cu * di.cus, std::max<uint32_t>(k, 1));
    }
    const size_t need = (size_t)n * slots;
    if (!p.dist || p.slot_elems < need) {
        BC_HIP_TRY(hipStreamSynchronize(st));
        for (void* q : {(void*)p.dist, (void*)p.sig, (void*)p.del})
            if (q) (void)hipFree(q);
        p.dist = nullptr;
        p.sig = p.del = nullptr;
        BC_HIP_TRY(hipMalloc((void**)&p.dist, need * sizeof(int32_t)));
        BC_HIP_TRY(hipMalloc((void**)&p.sig, need * sizeof(double)));
        BC_HIP_TRY(hipMalloc((void**)&p.del, need * sizeof(double)));
        p.slot_elems = need;
    }
    const unsigned zg = std::max(1u, std::min((n + 255) / 256, 4096u));
    hipLaunchKernelGGL(k_strat_zero, dim3(zg), dim3(256), 0, st, d_bc, n, p.words, 4u);
    BC_HIP_TRY(hipGetLastError());
    StratArgs a{};
    a.row_ptr = g.row_ptr;
    a.col = g.col;
    a.coo_src = p.coo_src;
    a.n = n;
    a.m = m;
    a.sources = d_sources;
    a.items = k;
    a.bc = d_bc;
    a.dist = p.dist;
    a.sig = p.sig;
    a.del = p.del;
    a.head = p.words;
    a.levels_max = p.words + 1;
    if (strategy != 3) {
        if (k > 0) {
            if (strategy == 1)
                hipLaunchKernelGGL(k_strategy_block<false>, dim3((unsigned)slots), dim3(wg), 0, st, a);
            else
                hipLaunchKernelGGL(k_strategy_block<true>, dim3((unsigned)slots), dim3(wg), 0, st, a);
            BC_HIP_TRY(hipGetLastError());
        }
        BC_HIP_TRY(hipMemcpyAsync(levels_max, p.words + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipStreamSynchronize(st));
        return;
    }
    // strategy 3: the host walks the sources and the levels
    std::vector<uint32_t> src(k);
    if (k > 0) {
        if (d_sources) {
            BC_HIP_TRY(hipMemcpyAsync(src.data(), d_sources, sizeof(uint32_t) * k, hipMemcpyDeviceToHost, st));
            BC_HIP_TRY(hipStreamSynchronize(st));
        } else {
            for (uint32_t i = 0; i < k; ++i) src[i] = i;
        }
    }
    int per_cu = 0;
    BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_strat_forward, wg, 0));
    const unsigned grid = (unsigned)std::max<long>(1, std::min<long>(((long)m + wg - 1) / wg, (long)std::max(per_cu, 1) * di.cus));
    uint32_t lmax = 0;
    for (uint32_t i = 0; i < k; ++i) {
        const uint32_t s = src[i];
        hipLaunchKernelGGL(k_strat_init, dim3(zg), dim3(256), 0, st, p.dist, p.sig, p.del, n, s);
        int d = 0;
        for (;;) {
            BC_HIP_TRY(hipMemsetAsync(p.words + 2, 0, sizeof(uint32_t), st));
            hipLaunchKernelGGL(k_strat_forward, dim3(grid), dim3(wg), 0, st, a, d, p.words + 2);
            BC_HIP_TRY(hipMemcpyAsync(p.h_flag, p.words + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            BC_HIP_TRY(hipStreamSynchronize(st));
            if (*p.h_flag == 0u) break;
            ++d;
        }
        for (int dd = d - 1; dd >= 0; --dd) hipLaunchKernelGGL(k_strat_backward, dim3(grid), dim3(wg), 0, st, a, dd);
        hipLaunchKernelGGL(k_strat_accumulate, dim3(zg), dim3(256), 0, st, p.del, d_bc, n, s);
        BC_HIP_TRY(hipGetLastError());
        lmax = std::max<uint32_t>(lmax, (uint32_t)(d + 1));
    }
    BC_HIP_TRY(hipStreamSynchronize(st));
    *levels_max = lmax;
}

}  // namespace bcmi
