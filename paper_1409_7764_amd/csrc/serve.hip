// Serving: BC requests on resident graphs, admitted by device-memory footprint and run by
// continuous batching.
//
// A server owns one HIP stream and one scheduler thread.  submit() only records the request
// (never touches the device).  The scheduler:
//   1. admits queued requests in arrival order while the summed footprint of admitted
//      requests stays within the budget (graph CSR+CSC, output, per-source state slots);
//   2. builds a "tick": round-robin over the admitted requests, each contributes its next
//      chunk of sources, so a request that arrives while others run joins the next tick and
//      small requests are not queued behind large ones;
//   3. launches the tick as one persistent launch per state home (LDS-resident for small
//      graphs, global-memory slots for the rest) over a work list that mixes requests and
//      graphs, plus one batched launch (64 sources per wavefront) per chunk of a request on
//      a larger, shallow graph; up to two ticks are queued on the stream so the device never
//      waits for the host;
//   4. when a tick's event has fired, requests whose last chunk it held are complete; their
//      device counters (copied back by the tick itself) fill the poll() record.
#include "bc_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

namespace bcmi {
struct Server;
namespace {

using Clock = std::chrono::steady_clock;

enum class RState { Queued, Admitted, Done, Failed };

struct Request {
    Graph* g = nullptr;
    std::vector<uint32_t> h_sources;   // sampled requests
    bool exact = false;
    uint32_t k = 0;                    // number of sources
    double* d_bc = nullptr;
    size_t footprint = 0;
    bool lds = false;
    bool batched = false;              // chunks run by the batched kernel
    RState state = RState::Queued;
    uint32_t* d_sources = nullptr;
    uint32_t* d_counters = nullptr;    // {done, overflowed, levels_max, bad}
    uint32_t* h_counters = nullptr;    // pinned copy, written by the completing tick
    uint32_t next = 0;                 // next source index to schedule
    uint32_t inflight = 0;             // chunks launched but not yet reaped
    double t_submit = 0, t_start = -1, t_done = -1;
    std::string error;
};

struct Chunk {
    uint64_t ticket;
    bool last;                         // this chunk completes the request
};

constexpr uint32_t kChunkGlobal = 64;     // sources per chunk on the global-slot path
constexpr uint32_t kChunkLds = 1024;      // sources per chunk on the LDS-resident path
constexpr uint32_t kChunkBatched = 16384;  // sources per chunk on the batched path (256 batches:
                                           // a launch carries ~1 ms of level-barrier latency, so
                                           // 1,024-source chunks ran at a third of the rate)
constexpr uint32_t kTickDescs = 4096;     // chunks per tick
constexpr uint32_t kTickBatched = 1;      // batched chunks per tick
constexpr int kServeTeams = 64;           // state slots of the batched path

struct Tick {
    bool busy = false;
    hipEvent_t done = nullptr;
    std::vector<Chunk> chunks;
    WorkDesc* h_desc = nullptr;        // pinned
    WorkDesc* d_desc = nullptr;
    CallStats* d_stats = nullptr;      // one per launch class
    uint32_t cap = 0;
    // batched chunks: two stats blocks each (batched launch, hand-off launch), the hand-off
    // launch's descriptor, and a flag raised when a batched team gave up at a barrier
    CallStats* d_bstats = nullptr;     // [2 * kTickBatched]
    WorkDesc* h_rdesc = nullptr;       // pinned [kTickBatched]
    WorkDesc* d_rdesc = nullptr;
    uint32_t* d_flag = nullptr;
    uint32_t* h_flag = nullptr;        // pinned
};

__global__ void k_zero_f64(double* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}
__global__ void k_zero_small(uint32_t* p, uint32_t n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0u;
}
__global__ void k_zero_stats(CallStats* s, uint32_t count) {
    uint32_t* w = reinterpret_cast<uint32_t*>(s);
    for (uint32_t i = threadIdx.x; i < count * (sizeof(CallStats) / 4); i += blockDim.x) w[i] = 0u;
}

// a batched chunk's counters into its request's {done, overflowed, levels_max, bad}
__global__ void k_fold_counters(const CallStats* b, const CallStats* h, uint32_t* counters, uint32_t* flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    counters[0] += b->n_done + h->n_done;
    counters[1] += b->n_overflow + h->n_overflow;
    counters[2] = max(counters[2], max(b->levels_max, h->levels_max));
    counters[3] += b->bad_source + h->bad_source;
    if (b->aborted) *flag = 1u;
}

// hand-off of a batched chunk's unfinished sources to the per-source kernel
struct HandOff {
    Server* s;
    const Request* r;
    CallStats* stats;
    WorkDesc* h_desc;
    WorkDesc* d_desc;
};
void serve_hand_off(void* ctx, const uint32_t* list, const uint32_t* count, uint32_t cap, bool kernel_ids,
                    hipStream_t st);

}  // namespace

struct Server {
    size_t budget = 0, used = 0;
    int max_slots = 0;
    int device = 0;
    hipStream_t st = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> active;
    std::unordered_map<uint64_t, Request> reqs;
    Clock::time_point t0;
    Knobs knobs;
    SlotPool pool;
    MsbPool* msb = nullptr;
    Tick ticks[2];
    std::string fatal;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

    size_t footprint(const Graph& g, uint32_t k, bool lds, bool batched) const {
        const size_t n = (size_t)g.n, m = g.m;
        size_t f = 2 * (4 * (n + 1) + 4 * m) + 8 * n;
        if (batched)
            f += (size_t)std::min<uint32_t>((k + 63) / 64, kServeTeams) *
                 msb_team_bytes((uint32_t)n, (uint32_t)std::min<uint64_t>(8 * n + 64, 0xffffffffull), 1024);
        else if (!lds)
            f += (size_t)std::min<uint32_t>(k, kChunkGlobal) * (24 * n + 4);
        return f;
    }

    void admit_locked() {
        while (!queue.empty()) {
            Request& r = reqs[queue.front()];
            if (used + r.footprint > budget) break;
            used += r.footprint;
            const uint32_t n = (uint32_t)r.g->n;
            BC_HIP_TRY(hipMalloc((void**)&r.d_counters, 4 * sizeof(uint32_t)));
            BC_HIP_TRY(hipHostMalloc((void**)&r.h_counters, 4 * sizeof(uint32_t), hipHostMallocDefault));
            if (!r.exact && r.k) {
                BC_HIP_TRY(hipMalloc((void**)&r.d_sources, sizeof(uint32_t) * r.k));
                BC_HIP_TRY(hipMemcpyAsync(r.d_sources, r.h_sources.data(), sizeof(uint32_t) * r.k,
                                          hipMemcpyHostToDevice, st));
            }
            hipLaunchKernelGGL(k_zero_f64, dim3(std::max(1u, std::min<unsigned>((n + 255) / 256, 1024))), dim3(256), 0,
                               st, r.d_bc, n);
            hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, st, r.d_counters, 4u);
            BC_HIP_TRY(hipGetLastError());
            if (r.k == 0) {   // nothing to run: done once the output is zeroed
                BC_HIP_TRY(hipStreamSynchronize(st));
                for (int i = 0; i < 4; ++i) r.h_counters[i] = 0;
                r.state = RState::Done;
                r.t_start = r.t_done = now_ms();
                used -= r.footprint;
                queue.pop_front();
                continue;
            }
            r.state = RState::Admitted;
            active.push_back(queue.front());
            queue.pop_front();
        }
    }

    bool has_schedulable_locked() const {
        for (uint64_t t : active) {
            const Request& r = reqs.at(t);
            if (r.next < r.k) return true;
        }
        return false;
    }

    // Builds and launches one tick from the admitted requests (lock held).
    void launch_tick_locked(Tick& tk) {
        std::vector<WorkDesc> cls[2];     // 0: LDS-resident, 1: global slots
        std::vector<Chunk> chunks[3];     // 2: batched
        uint32_t items[2] = {0, 0}, maxn[2] = {0, 0};
        // a tick holds about one round of the persistent grid, so its duration is bounded and a
        // request arriving meanwhile starts within roughly one source's search time
        const uint32_t item_cap[2] = {1u << 16, (uint32_t)std::max(1, max_slots)};
        struct BRun {
            uint64_t ticket;
            const uint32_t* sources;
            uint32_t take;
            bool last;
        };
        std::vector<BRun> bruns;
        bool progress = true;
        while (progress && cls[0].size() + cls[1].size() < kTickDescs) {
            progress = false;
            for (uint64_t t : active) {
                Request& r = reqs[t];
                if (r.next >= r.k) continue;
                if (r.batched) {   // one batched chunk per request and tick
                    if (bruns.size() >= kTickBatched) continue;
                    bool has = false;
                    for (const BRun& b : bruns) has |= b.ticket == t;
                    if (has) continue;
                    const uint32_t take = std::min(r.k - r.next, kChunkBatched);
                    // exact requests run the vertices in the graph's batching order
                    const uint32_t* src = r.exact ? r.g->order + r.next : r.d_sources + r.next;
                    r.next += take;
                    r.inflight += 1;
                    if (r.t_start < 0) r.t_start = now_ms();
                    bruns.push_back(BRun{t, src, take, r.next >= r.k});
                    progress = true;
                    continue;
                }
                const int c = r.lds ? 0 : 1;
                if (items[c] >= item_cap[c]) continue;
                const uint32_t take = std::min(r.k - r.next, r.lds ? kChunkLds : kChunkGlobal);
                WorkDesc d{};
                d.row_ptr = r.g->krow();
                d.col = r.g->kcol();
                d.perm = r.g->perm;
                d.iperm = r.g->iperm;
                d.bc = r.d_bc;
                d.sources = r.exact ? nullptr : r.d_sources + r.next;
                d.src_base = r.exact ? r.next : 0u;
                d.counters = r.d_counters;
                d.n = r.g->n;
                d.max_in = r.g->max_in_degree;
                d.item_begin = items[c];
                d.num_items = take;
                cls[c].push_back(d);
                r.next += take;
                r.inflight += 1;
                if (r.t_start < 0) r.t_start = now_ms();
                chunks[c].push_back(Chunk{t, r.next >= r.k});
                items[c] += take;
                maxn[c] = std::max(maxn[c], (uint32_t)r.g->n);
                progress = true;
                if (cls[0].size() + cls[1].size() >= kTickDescs) break;
            }
        }
        const size_t nd = cls[0].size() + cls[1].size();
        if (nd == 0 && bruns.empty()) return;
        if (nd) {
            for (size_t i = 0; i < cls[0].size(); ++i) tk.h_desc[i] = cls[0][i];
            for (size_t i = 0; i < cls[1].size(); ++i) tk.h_desc[cls[0].size() + i] = cls[1][i];
            BC_HIP_TRY(hipMemcpyAsync(tk.d_desc, tk.h_desc, sizeof(WorkDesc) * nd, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, st, tk.d_stats, 2u);
            BC_HIP_TRY(hipGetLastError());
        }
        for (int c = 0; c < 2; ++c) {
            if (cls[c].empty()) continue;
            Knobs k = knobs;
            if (c == 0) {   // LDS-resident graphs: the single-graph defaults for that path
                k.wg_size = 512;
                k.hub = 128;
            } else {
                k.lds_max_n = -1;
                k.teams = max_slots;
            }
            LaunchPlan p = make_plan(k, maxn[c], items[c], device);
            if (!p.lds_path) {
                if (!pool.rec || pool.slot_n < maxn[c] || pool.slots < (int)p.grid) {
                    pool_ensure(pool, std::max(maxn[c], pool.slot_n), std::max<int>(p.grid, pool.slots), st);
                }
                p.args.rec = pool.rec;
                p.args.queue = pool.queue;
                p.args.lvl = pool.lvl;
                p.args.slot_n = pool.slot_n;
            }
            p.args.descs = tk.d_desc + (c == 0 ? 0 : cls[0].size());
            p.args.ndesc = (uint32_t)cls[c].size();
            p.args.total_items = items[c];
            p.args.stats = tk.d_stats + c;
            p.args.zero_outputs = 0;   // outputs were zeroed at admission; requests span ticks
            enqueue_plan(p, st, 0);
        }
        // batched chunks after the per-source work of the tick, so small requests go first
        hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, st, tk.d_flag, 1u);
        for (size_t i = 0; i < bruns.size(); ++i) {
            const BRun& b = bruns[i];
            Request& r = reqs[b.ticket];
            CallStats* bs = tk.d_bstats + 2 * i;
            hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, st, bs, 2u);
            BC_HIP_TRY(hipGetLastError());
            HandOff h{this, &r, bs + 1, tk.h_rdesc + i, tk.d_rdesc + i};
            run_msb_enqueue(*msb, *r.g, b.sources, b.take, r.d_bc, bs, knobs.batch_wg, 0, kServeTeams, knobs.batch_pull,
                            st, serve_hand_off, &h);
            hipLaunchKernelGGL(k_fold_counters, dim3(1), dim3(1), 0, st, bs, bs + 1, r.d_counters, tk.d_flag);
            BC_HIP_TRY(hipGetLastError());
        }
        tk.chunks.clear();
        for (const BRun& b : bruns) chunks[2].push_back(Chunk{b.ticket, b.last});
        for (int c = 0; c < 3; ++c)
            for (const Chunk& ch : chunks[c]) {
                tk.chunks.push_back(ch);
                if (ch.last) {
                    Request& r = reqs[ch.ticket];
                    BC_HIP_TRY(hipMemcpyAsync(r.h_counters, r.d_counters, 4 * sizeof(uint32_t),
                                              hipMemcpyDeviceToHost, st));
                }
            }
        BC_HIP_TRY(hipMemcpyAsync(tk.h_flag, tk.d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipEventRecord(tk.done, st));
        tk.busy = true;
    }

    void reap_locked(Tick& tk) {
        const double t = now_ms();
        if (*tk.h_flag) {   // a batched team gave up waiting at a barrier: its state is dirty
            msb_pool_discard(msb);
            tk.chunks.clear();
            tk.busy = false;
            throw Error{BC_E_HIP, "batched launch: a team gave up waiting at a barrier"};
        }
        for (const Chunk& ch : tk.chunks) {
            auto it = reqs.find(ch.ticket);
            if (it == reqs.end()) continue;
            Request& r = it->second;
            r.inflight -= 1;
            if (r.inflight == 0 && r.next >= r.k && r.state == RState::Admitted) {
                r.state = RState::Done;
                r.t_done = t;
                used -= r.footprint;
                if (r.d_sources) (void)hipFree(r.d_sources);
                r.d_sources = nullptr;
                active.erase(std::find(active.begin(), active.end(), ch.ticket));
            }
        }
        tk.chunks.clear();
        tk.busy = false;
    }

    void fail_all_locked(const std::string& msg) {
        fatal = msg;
        for (auto& kv : reqs)
            if (kv.second.state == RState::Queued || kv.second.state == RState::Admitted) {
                kv.second.state = RState::Failed;
                kv.second.error = msg;
            }
        queue.clear();
        active.clear();
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            try {
                bool worked = false;
                for (Tick& tk : ticks)
                    if (tk.busy && hipEventQuery(tk.done) == hipSuccess) {
                        reap_locked(tk);
                        worked = true;
                    }
                if (!fatal.empty()) {
                    // nothing more runs after a device failure
                } else {
                    admit_locked();
                    for (Tick& tk : ticks)
                        if (!tk.busy && has_schedulable_locked()) {
                            launch_tick_locked(tk);
                            worked = true;
                        }
                }
                const bool idle = !ticks[0].busy && !ticks[1].busy;
                if (stopping && idle && (active.empty() || !fatal.empty())) break;
                if (!worked) {
                    if (idle && !has_schedulable_locked() && queue.empty()) cv.wait(lk);
                    else cv.wait_for(lk, std::chrono::microseconds(50));
                }
            } catch (const Error& e) {
                fail_all_locked(e.msg);
            } catch (const std::exception& e) {
                fail_all_locked(e.what());
            }
        }
    }
};

namespace {
void serve_hand_off(void* ctx, const uint32_t* list, const uint32_t* count, uint32_t cap, bool kernel_ids,
                    hipStream_t st) {
    HandOff& h = *reinterpret_cast<HandOff*>(ctx);
    Server& s = *h.s;
    const Graph& g = *h.r->g;
    Knobs k = s.knobs;
    k.lds_max_n = -1;
    k.teams = 64;
    LaunchPlan p = make_plan(k, (uint32_t)g.n, cap, s.device);
    if (!s.pool.rec || s.pool.slot_n < (uint32_t)g.n || s.pool.slots < (int)p.grid)
        pool_ensure(s.pool, std::max((uint32_t)g.n, s.pool.slot_n), std::max<int>(p.grid, s.pool.slots), st);
    p.args.rec = s.pool.rec;
    p.args.queue = s.pool.queue;
    p.args.lvl = s.pool.lvl;
    p.args.slot_n = s.pool.slot_n;
    WorkDesc d{};
    d.row_ptr = g.krow();
    d.col = g.kcol();
    d.bc = h.r->d_bc;
    d.sources = list;
    d.perm = kernel_ids ? nullptr : g.perm;
    d.iperm = g.iperm;
    d.n = g.n;
    d.max_in = g.max_in_degree;
    d.num_items = cap;
    *h.h_desc = d;   // pinned: stays valid until the tick completes
    BC_HIP_TRY(hipMemcpyAsync(h.d_desc, h.h_desc, sizeof(WorkDesc), hipMemcpyHostToDevice, st));
    p.args.descs = h.d_desc;
    p.args.ndesc = 1;
    p.args.total_items = 0;
    p.args.items_dev = count;   // the batched launch wrote how many sources it handed back
    p.args.stats = h.stats;
    p.args.zero_outputs = 0;
    enqueue_plan(p, st, 0);
}
}  // namespace

}  // namespace bcmi

using namespace bcmi;

namespace {
template <class F>
bc_status guarded_serve(F&& body) {
    try {
        clear_error();
        return body();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return BC_E_HIP;
    } catch (...) {
        set_error("unknown failure");
        return BC_E_HIP;
    }
}
}  // namespace

extern "C" {

bc_status bc_serve_create(size_t hbm_budget_bytes, int32_t max_slots, bc_server* out) {
    return guarded_serve([&]() -> bc_status {
        BC_REQUIRE(out != nullptr, BC_E_INVAL, "null output handle");
        BC_REQUIRE(hbm_budget_bytes > 0, BC_E_INVAL, "budget must be > 0");
        BC_REQUIRE(max_slots >= 0, BC_E_INVAL, "max_slots must be >= 0");
        Server* s = new Server();
        try {
            BC_HIP_TRY(hipGetDevice(&s->device));
            s->budget = hbm_budget_bytes;
            s->knobs = Knobs{};
            s->knobs.hub = 64;
            const DevInfo& di = dev_info(s->device);
            s->max_slots = max_slots > 0 ? max_slots : di.cus * 4;
            BC_HIP_TRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
            for (Tick& tk : s->ticks) {
                BC_HIP_TRY(hipEventCreateWithFlags(&tk.done, hipEventDisableTiming));
                BC_HIP_TRY(hipHostMalloc((void**)&tk.h_desc, sizeof(WorkDesc) * kTickDescs, hipHostMallocDefault));
                BC_HIP_TRY(hipMalloc((void**)&tk.d_desc, sizeof(WorkDesc) * kTickDescs));
                BC_HIP_TRY(hipMalloc((void**)&tk.d_stats, sizeof(CallStats) * 2));
                BC_HIP_TRY(hipMalloc((void**)&tk.d_bstats, sizeof(CallStats) * 2 * kTickBatched));
                BC_HIP_TRY(hipHostMalloc((void**)&tk.h_rdesc, sizeof(WorkDesc) * kTickBatched, hipHostMallocDefault));
                BC_HIP_TRY(hipMalloc((void**)&tk.d_rdesc, sizeof(WorkDesc) * kTickBatched));
                BC_HIP_TRY(hipMalloc((void**)&tk.d_flag, sizeof(uint32_t)));
                BC_HIP_TRY(hipHostMalloc((void**)&tk.h_flag, sizeof(uint32_t), hipHostMallocDefault));
                *tk.h_flag = 0;
                tk.cap = kTickDescs;
            }
            s->msb = msb_pool_new();
            s->t0 = Clock::now();
            s->th = std::thread([s] { s->loop(); });
        } catch (...) {
            delete s;
            throw;
        }
        *out = reinterpret_cast<bc_server>(s);
        return BC_OK;
    });
}

bc_status bc_serve_submit(bc_server sh, bc_graph gh, const uint32_t* h_sources, int32_t k, double* d_bc,
                          uint64_t* ticket) {
    return guarded_serve([&]() -> bc_status {
        BC_REQUIRE(sh && gh && d_bc && ticket, BC_E_INVAL, "null argument");
        Server* s = reinterpret_cast<Server*>(sh);
        Graph* g = reinterpret_cast<Graph*>(gh);
        BC_REQUIRE(g->device == s->device, BC_E_INVAL, "graph lives on another device");
        BC_REQUIRE(h_sources == nullptr || k >= 0, BC_E_INVAL, "k must be >= 0");
        Request r;
        r.g = g;
        r.exact = h_sources == nullptr;
        r.k = r.exact ? (uint32_t)g->n : (uint32_t)k;
        if (!r.exact) {
            r.h_sources.assign(h_sources, h_sources + k);
            for (uint32_t x : r.h_sources) BC_REQUIRE(x < (uint32_t)g->n, BC_E_RANGE, "source id >= n");
        }
        r.d_bc = d_bc;
        Knobs lds_knobs = s->knobs;
        lds_knobs.wg_size = 512;
        r.lds = lds_fits(lds_knobs, (uint32_t)g->n, s->device);
        // larger shallow graphs with at least one full batch of sources: 64 per wavefront
        r.batched = !r.lds && g->order && !g->deep && r.k >= 64 && s->knobs.batched >= 0;
        r.footprint = s->footprint(*g, r.k, r.lds, r.batched);
        BC_REQUIRE(r.footprint <= s->budget, BC_E_NOMEM, "request footprint exceeds the server budget");
        std::lock_guard<std::mutex> lk(s->mu);
        BC_REQUIRE(!s->stopping, BC_E_STATE, "server is stopping");
        BC_REQUIRE(s->fatal.empty(), BC_E_HIP, "server failed: " + s->fatal);
        r.t_submit = s->now_ms();
        const uint64_t t = s->next_ticket++;
        s->reqs.emplace(t, std::move(r));
        s->queue.push_back(t);
        *ticket = t;
        s->cv.notify_all();
        return BC_OK;
    });
}

bc_status bc_serve_poll(bc_server sh, uint64_t ticket, bc_info* info) {
    return guarded_serve([&]() -> bc_status {
        BC_REQUIRE(sh != nullptr, BC_E_INVAL, "null server");
        Server* s = reinterpret_cast<Server*>(sh);
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        BC_REQUIRE(it != s->reqs.end(), BC_E_STATE, "unknown ticket");
        const Request& r = it->second;
        if (r.state == RState::Failed) throw Error{BC_E_HIP, "request failed: " + r.error};
        if (r.state != RState::Done) return BC_PENDING;
        if (info) {
            bc_info o{};
            o.n_sources = r.h_counters[0];
            o.n_sigma_fp64_fallback = r.h_counters[1];
            o.levels_max = r.h_counters[2];
            o.path = r.batched ? 2u : (r.lds ? 1u : 0u);
            o.kernel_ms = r.t_done - r.t_start;
            o.t_submit_ms = r.t_submit;
            o.t_start_ms = r.t_start;
            o.t_done_ms = r.t_done;
            *info = o;
        }
        return BC_OK;
    });
}

bc_status bc_serve_destroy(bc_server sh) {
    return guarded_serve([&]() -> bc_status {
        BC_REQUIRE(sh != nullptr, BC_E_INVAL, "null server");
        Server* s = reinterpret_cast<Server*>(sh);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
            for (uint64_t t : s->queue) s->reqs[t].state = RState::Failed;   // never admitted: cancelled
            s->queue.clear();
            s->cv.notify_all();
        }
        if (s->th.joinable()) s->th.join();
        (void)hipStreamSynchronize(s->st);
        for (auto& kv : s->reqs) {
            if (kv.second.d_sources) (void)hipFree(kv.second.d_sources);
            if (kv.second.d_counters) (void)hipFree(kv.second.d_counters);
            if (kv.second.h_counters) (void)hipHostFree(kv.second.h_counters);
        }
        for (Tick& tk : s->ticks) {
            if (tk.done) (void)hipEventDestroy(tk.done);
            if (tk.h_desc) (void)hipHostFree(tk.h_desc);
            if (tk.d_desc) (void)hipFree(tk.d_desc);
            if (tk.d_stats) (void)hipFree(tk.d_stats);
            if (tk.d_bstats) (void)hipFree(tk.d_bstats);
            if (tk.h_rdesc) (void)hipHostFree(tk.h_rdesc);
            if (tk.d_rdesc) (void)hipFree(tk.d_rdesc);
            if (tk.d_flag) (void)hipFree(tk.d_flag);
            if (tk.h_flag) (void)hipHostFree(tk.h_flag);
        }
        pool_free(s->pool);
        msb_pool_delete(s->msb);
        (void)hipStreamDestroy(s->st);
        delete s;
        return BC_OK;
    });
}

}  // extern "C"
