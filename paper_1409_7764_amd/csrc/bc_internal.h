// Internal declarations shared by the HIP translation units of libbcmi.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bc.h"

namespace bcmi {

// ---------------------------------------------------------------------------------------
// error plumbing: every ABI entry point converts failures into a status + message
// ---------------------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Error {
    bc_status code;
    std::string msg;
};

#define BC_HIP_TRY(expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            throw ::bcmi::Error{e_ == hipErrorOutOfMemory ? BC_E_NOMEM : BC_E_HIP,              \
                                std::string(#expr) + ": " + hipGetErrorString(e_)};             \
    } while (0)

#define BC_REQUIRE(cond, code, msg)                                                             \
    do {                                                                                        \
        if (!(cond)) throw ::bcmi::Error{(code), (msg)};                                        \
    } while (0)

// ---------------------------------------------------------------------------------------
// device-side per-vertex record of one source's search.
//   dist : BFS level, -1 = not reached
//   val  : forward sweep  -> shortest-path count (uint64 bits, or double bits after overflow)
//          backward sweep -> psi = (1 + delta) / sigma (double bits), once the vertex's
//                            level has been finished
// Keeping dist and the count in one 16-byte record means the count update of a DAG edge
// touches the cache line the distance test has just fetched.
// ---------------------------------------------------------------------------------------
struct alignas(16) VRec {
    int32_t dist;
    uint32_t pad;
    uint64_t val;
};

// Per-call device counters (written by the kernels, read back for bc_info).
struct CallStats {
    uint32_t work_head;      // next work item to claim
    uint32_t n_done;         // sources completed
    uint32_t n_overflow;     // sources recounted in double precision
    uint32_t levels_max;     // deepest search
    uint32_t bad_source;     // sources with id >= n (skipped)
    uint32_t work_head2;     // work counter of a follow-up launch in the same call
    uint32_t aborted;        // a batched team gave up waiting at a barrier
    uint32_t handoffs;       // batched and deep-graph paths: sources handed to the global-memory kernel
    uint64_t reached;        // sum over sources of reached vertices (source included)
    uint64_t examined;       // sum over sources of out-edges of reached vertices
    uint64_t dag_edges;      // sum over sources of shortest-path DAG edges
    uint64_t entries;        // batched path: (vertex, level) entries of the batches' level lists
    uint64_t edge_visits;    // batched path: out-edges read per entry (once per sweep)
    uint64_t scans;          // batched path: level-collect passes over all vertices
    uint64_t cycles[3];      // batched path: workgroup clock cycles in forward, backward, reset
    uint64_t pull_edges;     // batched path: in-edges read by pulled levels
    uint64_t pull_levels;    // batched path: levels pulled (summed over batches)
    uint64_t pull_skip;      // batched path: out-edges of the entries of pulled levels (not pushed)
    uint64_t pull_pairs;     // batched path: DAG (edge, source) pairs found by pulled levels
};

// Launch knobs after defaults / tuning are applied.
struct Knobs {
    int wg_size = 256;
    int team = 0;                // batched path: workgroups per batch (0 = from the batch count)
    int teams = 0;               // concurrent sources; 0 = fill the device
    int hub = 32;                // wavefront-per-vertex threshold
    int lds_max_n = 4096;
    bool use_graph = true;
    int batched = 0;             // 1: 64-source batches, -1: one source per workgroup, 3: one source per
                                 // workgroup with its levels in LDS tables, 0: auto (2: rejected)
    int batch_wg = 512;          // workgroup size of the batched kernel
    int batch_pull = 32;         // batched path: pull a level when (in-edges of unreached vertices) * 16 <
                                 // (out-edges of the level) * batch_pull; <= 0 = never
    bool deterministic = false;  // fixed summation order (global-memory kernel, per-workgroup partials)
};

// Graph handle (the opaque bc_graph).
struct Graph {
    Graph();
    int device = 0;
    // identity that is never reused within the process (a handle's address can be, once it is
    // freed): cached launch plans are keyed by it
    uint64_t uid = 0;
    int32_t n = 0;
    uint32_t m = 0;
    uint32_t* row_ptr = nullptr;   // n+1
    uint32_t* col = nullptr;       // m
    uint32_t* csc_ptr = nullptr;   // n+1
    uint32_t* csc_row = nullptr;   // m
    // the kernels run on a copy with vertices relabelled by decreasing in-degree (graphs of
    // at least kRelabelMinN vertices): the most often gathered targets then share cache lines
    uint32_t* perm = nullptr;      // caller id -> kernel id (null: identity)
    uint32_t* iperm = nullptr;     // kernel id -> caller id
    uint32_t* prow = nullptr;      // kernel CSR (n+1), successors sorted per row
    uint32_t* pcol = nullptr;      // m
    // batching order of the batched path (caller ids): rank[v] = position of v in `order`,
    // vertices with out-edges first (null when not built)
    uint32_t* rank = nullptr;      // n
    uint32_t* order = nullptr;     // n
    // fewer than half of the vertices with out-edges lie within the ranked levels of the
    // batching order: a deep graph (lattice-like), run one source per workgroup by default
    bool deep = false;
    const uint32_t* krow() const { return prow ? prow : row_ptr; }
    const uint32_t* kcol() const { return pcol ? pcol : col; }
    uint32_t max_out_degree = 0;
    uint32_t max_in_degree = 0;
    uint32_t zero_out_degree = 0;  // vertices with no out-edges (sources that reach nothing)
    // per-source scratch, grown on demand and reused between calls
    void* slots = nullptr;
    struct StratPool* strat = nullptr;   // state of the paper's strategy baselines
    CallStats* stats = nullptr;    // device
    std::mutex mu;
    ~Graph();
};

// Device properties used for launch sizing.
struct DevInfo {
    int cus = 256;
    int lds_per_block = 65536;
    int lds_per_cu = 163840;
    int max_threads = 1024;
    std::string name;
};
const DevInfo& dev_info(int device);

constexpr int32_t kRelabelMinN = 16384;

// ---- CSR builder (csr_build.hip) --------------------------------------------------------
void build_csr_device(int32_t n, int64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                      hipStream_t stream, Graph& g);

// ---- per-source kernels (bc_kernels.hip) -------------------------------------------------
struct RunArgs {
    const Graph* g;
    const uint32_t* sources;   // nullable: item i is source i
    uint32_t num_items;
    double* bc;                // nullable (bc_sssp)
    uint8_t* ovf_flags = nullptr;   // nullable: per-source overflow flags by caller id (n bytes)
    // optional export of one source's arrays (bc_sssp)
    int32_t* ex_dist = nullptr;
    uint64_t* ex_sigma = nullptr;
    double* ex_sigma_f = nullptr;
    double* ex_delta = nullptr;
};
// Enqueue a full BC pass over the given sources on `stream` (zeroes bc first).  Returns
// which path ran (0 global slots, 1 LDS, 2 batched, 3 levels in LDS).
int run_sources(const RunArgs& a, const Knobs& k, hipStream_t stream, Graph& g);
void read_stats(Graph& g, hipStream_t stream, CallStats* out);

// ---- launch plumbing shared by the single-graph, batch and serving paths ------------------
// One descriptor per (graph, source range) of a launch's work list.
struct WorkDesc {
    const uint32_t* row_ptr;
    const uint32_t* col;
    double* bc;
    const uint32_t* sources;   // nullable: local item i is source src_base + i (kernel ids)
    const uint32_t* perm;      // nullable: caller id -> kernel id, applied to `sources`
    const uint32_t* iperm;     // nullable: kernel id -> caller id, applied to every output index
    uint32_t* counters;        // nullable: per-descriptor {done, overflowed, levels_max, bad}
    uint8_t* ovf_flags;        // nullable: n bytes by caller id, 1 where a source of the launch was
                               // recounted in double precision (zeroed with the BC output)
    int32_t n;
    uint32_t max_in;           // largest in-degree (bounds the counts; 0 = unknown)
    uint32_t item_begin;       // first work item of this descriptor in the launch
    uint32_t num_items;
    uint32_t src_base;
};

struct LaunchArgs {
    const WorkDesc* descs;
    uint32_t ndesc;
    uint32_t total_items;
    CallStats* stats;
    uint32_t hub;
    uint32_t tpv_max;          // chunk max degree up to which thread-per-vertex is used
    // global-memory slots
    VRec* rec;
    uint32_t* queue;
    uint32_t* lvl;
    uint32_t slot_n;
    uint32_t lds_n;            // LDS path: vertex capacity
    uint32_t zero_outputs;     // zero each descriptor's BC output and counters first
    const uint32_t* items_dev; // nullable: number of work items, read on the device
    uint32_t* head;            // nullable: work counter (default: stats->work_head)
    // export of one source (inspection entry point)
    int32_t* ex_dist;
    uint64_t* ex_sigma;
    double* ex_sigma_f;
    double* ex_delta;
    // deterministic mode (global-memory kernel): workgroup b takes items b, b + grid, ... in
    // order and adds its dependencies into part + b * n (plain adds); a fixed-order reduction
    // over the workgroups writes BC
    double* part;
    uint32_t det;
};

// Device-resident per-source state slots of the global-memory path.
struct SlotPool {
    VRec* rec = nullptr;
    uint32_t* queue = nullptr;
    uint32_t* lvl = nullptr;
    uint32_t slot_n = 0;
    int slots = 0;
};

// One persistent launch over a device-resident work list.
struct LaunchPlan {
    bool lds_path = false;
    int wg = 256;
    unsigned grid = 0;
    size_t dyn_lds = 0;
    LaunchArgs args{};
};

LaunchPlan make_plan(const Knobs& k, uint32_t max_n, uint32_t items, int device);
WorkDesc single_graph_desc(const Graph& g, const RunArgs& ra);
void store_desc(WorkDesc* dst, const WorkDesc& d, hipStream_t st);
void reset_slot_records(VRec* rec, size_t count, hipStream_t st);
void enqueue_plan(const LaunchPlan& p, hipStream_t st, uint32_t max_n);
void pool_ensure(SlotPool& p, uint32_t slot_n, int slots, hipStream_t st);
void pool_free(SlotPool& p);
size_t pool_bytes(uint32_t slot_n, int slots);
bool lds_fits(const Knobs& k, uint32_t n, int device);

// ---- 64 sources per batch (msb.hip) ---------------------------------------------------------
struct MsbPool;
MsbPool* msb_pool_new();
void msb_pool_delete(MsbPool* p);
void msb_pool_discard(MsbPool* p);
size_t msb_team_bytes(uint32_t n, uint32_t cap, uint32_t max_levels);
// enqueues the per-source launch over the sources a batched launch hands back: (ctx, list,
// device count, capacity, list holds kernel ids, stream)
using RetryLaunch = void (*)(void*, const uint32_t*, const uint32_t*, uint32_t, bool, hipStream_t);
void run_msb_enqueue(MsbPool& p, const Graph& g, const uint32_t* sources, uint32_t k, double* bc, CallStats* stats,
                     int wg, int team_knob, int slots_cap, int pull16, hipStream_t st, RetryLaunch retry_launch,
                     void* retry_ctx);

// ---- one source per workgroup, levels in LDS hash tables (deep.hip) ----------------------
struct DeepPool;
DeepPool* deep_pool_new();
void deep_pool_delete(DeepPool* p);
size_t deep_slot_bytes(uint32_t n);
void deep_geometry(int device, uint32_t& H, uint32_t& F, size_t& dyn);
// sources given in caller numbering (null: item i is source i); sources whose levels outgrow
// the LDS tables are handed to `retry_launch` with caller ids
void run_deep_enqueue(DeepPool& p, const Graph& g, const uint32_t* sources, uint32_t k, double* bc,
                      uint8_t* ovf_flags, CallStats* stats, int slots_cap, hipStream_t st, RetryLaunch retry_launch,
                      void* retry_ctx);

// ---- the paper's three strategies as baselines (strategies.hip) ---------------------------
void strat_pool_delete(StratPool* p);
// strategy 1 vertex-parallel / 2 edge-parallel (one workgroup per source), 3 edge-parallel over
// the grid with host-synchronised levels; sources in caller ids (null: all n); zeroes d_bc
void run_strategy(StratPool*& pool, const Graph& g, int strategy, int wg, const uint32_t* d_sources, uint32_t k,
                  double* d_bc, hipStream_t st, uint32_t* levels_max);

// ---- approximate BC by source sampling (approx.hip) ------------------------------------------
void draw_pivots(uint64_t seed, uint32_t n, uint32_t k, uint32_t* out);   // SplitMix64, uniform on [0, n)
uint32_t hoeffding_pivots(uint32_t n, double eps, double delta);        // n when the bound needs >= n
void scale_bc(double* d_bc, uint32_t n, double f, hipStream_t st);
double read_bc_entry(const double* d_bc, uint32_t v, double* d_tmp, hipStream_t st);

// ---- sampled BC with the state in the library's fixed per-device array (noalloc.hip) ---------
void run_sampled_noalloc(Graph& g, const uint32_t* sources, uint32_t k, double* bc, const Knobs& kn, hipStream_t st);
uint32_t noalloc_max_n();

// ---- STREAM-style bandwidth probe (stream_probe.hip) -------------------------------------------
void stream_probe(size_t bytes, int reps, double* copy_gbs, double* triad_gbs);

// ---- tuning (tune.hip) -------------------------------------------------------------------
Knobs resolve_knobs(Graph& g, const bc_tuning* t);
Knobs default_knobs(const Graph& g);
bool tuning_enabled();

}  // namespace bcmi
