// Deep-graph path: one source per workgroup, each BFS level held in LDS hash tables (the
// device code, with its layout and the method's steps, is in deep_kernel.h).  This file holds
// the launch: LDS geometry, the per-slot global state, and the hand-off of sources whose levels
// outgrow the tables to the global-memory kernel.
#include "bc_internal.h"
#include "deep_kernel.h"

#include <algorithm>

namespace bcmi {

namespace {

__global__ void __launch_bounds__(deep::kWG) k_bc_deep(deep::Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    deep::worker<deep::kWG>(a, smem);
}

}  // namespace

struct DeepPool {
    uint8_t* seen = nullptr;
    uint32_t* lv = nullptr;
    uint32_t* lb = nullptr;
    uint32_t* ld = nullptr;
    uint64_t* ls = nullptr;
    uint32_t* lvl = nullptr;
    uint32_t* retry = nullptr;
    uint32_t n = 0;
    size_t seen_stride = 0, list_stride = 0, lvl_stride = 0;
    int slots = 0;
    uint32_t retry_cap = 0;
};

DeepPool* deep_pool_new() { return new DeepPool(); }

static void deep_pool_release(DeepPool& p) {
    for (void* q : {(void*)p.seen, (void*)p.lv, (void*)p.lb, (void*)p.ld, (void*)p.ls, (void*)p.lvl})
        if (q) (void)hipFree(q);
    p.seen = nullptr;
    p.lv = p.lb = p.ld = p.lvl = nullptr;
    p.ls = nullptr;
    p.n = 0;
    p.slots = 0;
}

void deep_pool_delete(DeepPool* p) {
    if (!p) return;
    deep_pool_release(*p);
    if (p->retry) (void)hipFree(p->retry);
    delete p;
}

// device bytes of one slot: reached bytes, the level lists (vertex, CSR begin, out-degree,
// count) and the first entry of each level
size_t deep_slot_bytes(uint32_t n) {
    return (((size_t)n + 255) & ~(size_t)255) + (size_t)n * (4 + 4 + 4 + 8) + ((size_t)n + 2) * 4;
}

// LDS geometry: H hash slots per table (a multiple of 64), the largest for which two
// workgroups share a compute unit; a level holds at most F = H/2 vertices
void deep_geometry(int device, uint32_t& H, uint32_t& F, size_t& dyn) {
    const DevInfo& di = dev_info(device);
    const size_t per_wg = std::min<size_t>((size_t)di.lds_per_cu / 2, (size_t)di.lds_per_block);
    const size_t fixed = deep::lds_bytes(0) + 512;   // control words, allocation granule
    const size_t room = per_wg > fixed ? per_wg - fixed : 0;
    uint32_t h = (uint32_t)(room / 42) / 64 * 64;    // 40 B per slot in the two tables, 4 B per listed vertex
    H = std::max<uint32_t>(h, 128);
    F = H / 2;
    dyn = deep::lds_bytes(H);
}

void run_deep_enqueue(DeepPool& p, const Graph& g, const uint32_t* sources, uint32_t k, double* bc,
                      uint8_t* ovf_flags, CallStats* stats, int slots_cap, hipStream_t st, RetryLaunch retry_launch,
                      void* retry_ctx) {
    if (k == 0) return;
    uint32_t H, F;
    size_t dyn;
    deep_geometry(g.device, H, F, dyn);
    BC_HIP_TRY(hipFuncSetAttribute((const void*)k_bc_deep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    int per_cu = 0;
    BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bc_deep, deep::kWG, dyn));
    BC_REQUIRE(per_cu >= 1, BC_E_HIP, "deep-graph kernel does not fit on a compute unit");
    long grid = (long)per_cu * dev_info(g.device).cus;
    if (slots_cap > 0) grid = std::min<long>(grid, slots_cap);
    grid = std::min<long>(grid, k);
    const uint32_t n = (uint32_t)g.n;
    if (!p.seen || p.n < n || p.slots < grid) {
        BC_HIP_TRY(hipStreamSynchronize(st));
        deep_pool_release(p);
        size_t free_b = 0, total_b = 0;
        BC_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        const long fit = (long)((free_b / 2) / deep_slot_bytes(n));
        BC_REQUIRE(fit >= 1, BC_E_NOMEM, "no room for one deep-graph slot");
        const int slots = (int)std::min<long>(grid, fit);
        p.seen_stride = ((size_t)n + 255) & ~(size_t)255;
        p.list_stride = n;
        p.lvl_stride = (size_t)n + 2;
        BC_HIP_TRY(hipMalloc((void**)&p.seen, p.seen_stride * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.lv, p.list_stride * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.lb, p.list_stride * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.ld, p.list_stride * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.ls, p.list_stride * 8 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.lvl, p.lvl_stride * 4 * slots));
        BC_HIP_TRY(hipMemsetAsync(p.seen, 0, p.seen_stride * slots, st));
        p.n = n;
        p.slots = slots;
    }
    grid = std::min<long>(grid, p.slots);
    if (p.retry_cap < k) {
        BC_HIP_TRY(hipStreamSynchronize(st));
        if (p.retry) (void)hipFree(p.retry);
        p.retry = nullptr;
        BC_HIP_TRY(hipMalloc((void**)&p.retry, (size_t)k * 4));
        p.retry_cap = k;
    }
    deep::Args a{};
    a.row_ptr = g.row_ptr;   // caller numbering: a deep graph's own ids keep its locality
    a.col = g.col;
    a.bc = bc;
    a.ovf_flags = ovf_flags;
    a.sources = sources;
    a.n = n;
    a.items = k;
    a.H = H;
    a.F = F;
    a.work_head = &stats->work_head;
    a.handoffs = &stats->handoffs;
    a.bad_source = &stats->bad_source;
    a.retry = p.retry;
    a.reached = &stats->reached;
    a.examined = &stats->examined;
    a.dag_edges = &stats->dag_edges;
    a.n_done = &stats->n_done;
    a.n_overflow = &stats->n_overflow;
    a.levels_max = &stats->levels_max;
    a.seen = p.seen;
    a.seen_stride = p.seen_stride;
    a.lv = p.lv;
    a.lb = p.lb;
    a.ld = p.ld;
    a.ls = p.ls;
    a.list_stride = p.list_stride;   // a pool built for a larger graph keeps its strides
    a.lvl = p.lvl;
    a.lvl_stride = p.lvl_stride;
    BC_REQUIRE(p.list_stride >= n && p.lvl_stride >= (size_t)n + 1 && p.seen_stride >= n && grid <= p.slots,
               BC_E_HIP, "deep-graph slot pool smaller than the launch");
    hipLaunchKernelGGL(k_bc_deep, dim3((unsigned)grid), dim3(deep::kWG), dyn, st, a);
    BC_HIP_TRY(hipGetLastError());
    // sources whose levels outgrew the tables: the global-memory kernel, same stream
    retry_launch(retry_ctx, p.retry, &stats->handoffs, k, false, st);
}

}  // namespace bcmi
