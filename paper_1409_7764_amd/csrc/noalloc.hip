// Sampled BC without any device allocation, for callers that cannot allocate (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The computation is bc_sampled's one-source-per-workgroup path with the per-source state in
// global memory (section I's forward and backward sweeps, the same kernel), but every buffer
// beyond the caller's inputs and outputs lives in one fixed array of device memory that the
// library holds per GPU for the life of the process:
//   [0, 256)        the launch's work descriptor
//   [256, 512)      the call's counters
//   then            per-source state slots: records {dist, count}, BFS queue, level offsets
// The number of slots is what fits (at most one per resident workgroup); a graph whose single
// slot does not fit is rejected.  Every call on a device shares its array and leaves it dirty:
// each call rewrites the descriptor, zeroes the counters and resets every slot record before
// its search, and calls that overlap on one device race on the array.
#include "bc_internal.h"

#include <algorithm>

namespace bcmi {

namespace {

constexpr size_t kScratchBytes = 32ull << 20;   // 32 MiB per device
constexpr size_t kHeadBytes = 512;              // descriptor + counters
constexpr int kMaxDevices = 64;

// The array itself.  In host code this name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

unsigned char* scratch_on(int dev) {
    BC_REQUIRE(dev >= 0 && dev < kMaxDevices, BC_E_HIP, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {   // first call on this device, with the device current
        void* p = nullptr;
        BC_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        BC_REQUIRE(p != nullptr, BC_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = reinterpret_cast<unsigned char*>(p);
    }
    return g_scratch_ptr[dev];
}

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes of `slots` slots for graphs of n vertices, after the head
size_t slots_bytes(size_t n, size_t slots) {
    return up256(slots * n * sizeof(VRec)) + up256(slots * n * 4) + up256(slots * (n + 1) * 4);
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Largest n with one slot inside the array.
uint32_t noalloc_max_n() {
    size_t lo = 1, hi = kScratchBytes;   // slots_bytes(n, 1) grows with n
    while (lo < hi) {
        const size_t mid = (lo + hi + 1) / 2;
        if (kHeadBytes + slots_bytes(mid, 1) <= kScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return (uint32_t)lo;
}

void run_sampled_noalloc(Graph& g, const uint32_t* sources, uint32_t k, double* bc, const Knobs& kn,
                         hipStream_t st) {
    const uint32_t n = (uint32_t)g.n;
    const uint32_t max_n = noalloc_max_n();
    BC_REQUIRE(n <= max_n, BC_E_RANGE,
               "graph too large for the allocation-free entry point: n must be <= " + std::to_string(max_n) +
                   " (one state slot in its " + std::to_string(kScratchBytes >> 20) + " MiB array)");
    int dev = 0;
    BC_HIP_TRY(hipGetDevice(&dev));
    BC_REQUIRE(dev == g.device, BC_E_INVAL, "graph lives on another device");
    unsigned char* base = scratch_on(dev);
    WorkDesc* d_desc = reinterpret_cast<WorkDesc*>(base);
    CallStats* d_stats = reinterpret_cast<CallStats*>(base + 256);
    static_assert(sizeof(WorkDesc) <= 256 && sizeof(CallStats) <= 256, "head of the scratch array too small");

    // one source per workgroup, state in global memory (the LDS-resident path needs no slots,
    // but this entry point keeps to one kernel)
    Knobs k2 = kn;
    k2.lds_max_n = -1;
    LaunchPlan p = make_plan(k2, n, k, g.device);
    size_t slots = std::max<size_t>(1, p.grid);
    while (slots > 1 && kHeadBytes + slots_bytes(n, slots) > kScratchBytes) --slots;
    p.grid = (unsigned)std::min<size_t>(p.grid, slots);

    unsigned char* q = base + kHeadBytes;
    VRec* rec = reinterpret_cast<VRec*>(q);
    q += up256(slots * (size_t)n * sizeof(VRec));
    uint32_t* queue = reinterpret_cast<uint32_t*>(q);
    q += up256(slots * (size_t)n * 4);
    uint32_t* lvl = reinterpret_cast<uint32_t*>(q);

    RunArgs ra{};
    ra.g = &g;
    ra.sources = sources;
    ra.num_items = k;
    ra.bc = bc;
    store_desc(d_desc, single_graph_desc(g, ra), st);
    reset_slot_records(rec, slots * (size_t)n, st);   // the last call left its own layout behind
    p.args.rec = rec;
    p.args.queue = queue;
    p.args.lvl = lvl;
    p.args.slot_n = n;
    p.args.descs = d_desc;
    p.args.ndesc = 1;
    p.args.total_items = k;
    p.args.stats = d_stats;
    enqueue_plan(p, st, n);   // zeroes the counters and the output, then the persistent search
}

}  // namespace bcmi
