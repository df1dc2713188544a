// Brandes betweenness centrality with 64 sources per batch, one source per wavefront lane.
//
// The forward and backward sweeps of section I's method are run for a batch of up to 64
// sources at once.  A vertex v enters the level-d list of the batch once, with the bit mask
// of the batch's sources for which d(s, v) = d; an out-edge of v is therefore read once per
// level for all of those sources.  Per-(vertex, source) state lives in 64-wide rows, so the
// per-source updates of one edge are one coalesced row access instead of 64 scattered ones:
//   seen[v]     sources that reached v at a level <= d         (64-bit mask)
//   nxt[v]      sources reaching v at level d+1 (forward)
//               (seen and nxt of a vertex share one 16-byte record: one gather per edge)
//   bnx[v]      backward sweep: the level-(d+1) masks, scattered into a dense 8-byte array
//               (twice as many vertices per cache line as the records; seen is not needed)
//   sig[v][s]   shortest-path count sigma_s(v) (uint32: a 256-byte row)
//   psi[v][s]   psi_s(v) = (1 + delta_s(v)) / sigma_s(v) (double), written when the backward
//               sweep finishes v's level
//
// forward, level d, entry (v, f): for each successor w the lanes of one wavefront test 64
//   edges at once: dag = f & ~seen[w] are the sources with w at level d+1; they are OR-ed
//   into nxt[w] and, lane per source, sig[w][s] += sig[v][s] for s in dag (32-bit integer
//   atomics, never waiting for the old value).  sigma_s(w) is at most in-degree(w) times the
//   largest sigma_s on level d, so a lane whose sigma_s(v) times the largest in-degree reaches
//   2^32 is flagged before its sums can wrap; the per-source kernel recounts that source
//   (64-bit counts, then double precision).  No operation of the expansion waits for a
//   returned value, and a wavefront runs two units at
//   a time, so a pair of units costs two dependent memory round trips.  The level-(d+1) list
//   is then collected by one coalesced pass over nxt (entries in vertex order), which also
//   folds the masks into seen.
// pulled levels (direction-optimising forward): when the vertices that some source of the batch
//   has not reached have fewer in-edges than the level's entries have out-edges, level d + 1 is
//   built from the other side.  Every vertex w with unreached lanes u(w) reads its in-edges
//   (CSC) and the level-d lanes cur[x] of each in-neighbour x; lane s sums sigma_s(x) over the
//   in-neighbours whose lanes hold s, and w stores its own row and next-mask: no count atomics,
//   and only the in-edges of unreached vertices are read (late levels, where most out-edges of
//   a wide frontier lead back into reached vertices).  The same cap on the summed counts flags
//   a lane before any sum can wrap.  The backward sweep does not depend on the direction.
// backward, level d, entry (v, f): succ = f & nxt[w] are the sources with w one level down;
//   lane s sums psi_s(w), then delta_s(v) = sigma_s(v) * sum, psi_s(v) is stored, and sum
//   over s != v of delta_s(v) is added to BC[v].  Each (v, s) has one
//   owner lane: no atomics on delta.  A vertex with more than 64 out-edges is split into
//   pieces; their partial sums meet in a per-batch accumulator row before the owner
//   finishes the vertex.
//
// Sources are batched in the graph's batching order (built with the CSR: vertices ranked
// outward from a hub over reversed edges, grouped by the successor through which they reach
// it).  Sources batched that way share most of their DAG edges and reach vertices at the same
// levels, so a row update carries more sources and touches fewer sectors of the row.  Sources
// without out-edges reach no vertex and contribute nothing, so they are not run.
#include "bc_internal.h"

#include <algorithm>
#include <atomic>

namespace bcmi {

// Per-team control block in global memory (a team = the workgroups sharing one batch).
struct alignas(128) TeamCtl {
    uint32_t bar_count;
    uint32_t bar_gen;
    uint32_t batch;          // batch being run
    uint32_t tail;           // level-list append position
    uint32_t cc;             // chunk claim counter of the current phase
    uint32_t abort;          // a barrier wait ran out: every member leaves
    uint32_t sdeg[2];        // out-degree sum of a level (double-buffered by level parity)
    uint64_t ovf;            // sources whose counts carried out of 64 bits
    uint32_t pin[2];         // in-edges of vertices some source has not reached yet, by level parity
    uint32_t pad[14];
};

struct MsbArgs {
    const uint32_t* row_ptr;     // kernel CSR
    const uint32_t* col;
    double* bc;                  // caller's output, indexed through iperm
    const uint32_t* iperm;       // nullable: kernel id -> caller id
    const uint32_t* plan;        // planned sources, batched in order
    const uint32_t* plan_count;  // [0]: number of planned sources
    uint32_t* retry;             // sources handed to the per-source kernel
    uint32_t* retry_count;
    CallStats* stats;
    TeamCtl* ctl;                // [teams]
    uint64_t* masks;             // [teams][n][2]: {seen, nxt} per vertex
    uint32_t* sig;               // [teams][n][64] counts
    double* psi;                 // [teams][n][64]
    double* hacc;                // [workgroups][hub_rows][64], accumulator rows beyond the LDS ones
    double* bcp;                 // [teams][cap]: each list entry's BC contribution
    uint32_t* lst_v;             // [teams][cap]
    uint64_t* lst_m;             // [teams][cap]
    uint32_t* lvl;               // [teams][max_levels + 2]
    int32_t n;
    uint64_t mask_stride;        // elements between two teams' mask arrays
    uint64_t sig_stride;         // elements between two teams' count rows
    uint64_t psi_stride;         // elements between two teams' psi rows
    uint32_t cap;
    uint32_t max_levels;
    uint32_t hub_rows;
    uint32_t team_size;          // workgroups per team; 0 = as many as the batch count allows
    uint32_t pool_teams;         // team slots in the pool
    uint32_t sig_cap;            // largest count c with c * (largest in-degree) < 2^32
    uint64_t* bnx;               // [teams][n]: backward sweep, level-(d+1) masks; zero between batches
    uint64_t bnx_stride;
    const uint32_t* csc_ptr;     // pulled levels: in-edges of each vertex
    const uint32_t* csc_row;
    ulonglong2* cur;             // [teams][n]: {lanes on level d, d + 1} of the vertices listed on level d;
                                 // zero between batches
    uint64_t cur_stride;
    uint64_t wait_ticks;         // wall-clock ticks a barrier waits before the team gives up
    uint32_t pull16;             // a level is pulled when (in-edges of vertices with unreached lanes) * 16 <
                                 // (out-edges of the level's entries) * pull16; 0 = never
};

namespace {

// A team gives up waiting at a barrier after MsbArgs::wait_ticks of the constant-rate wall clock
// (set by the host from the graph's size: far above what any level of that graph takes).
// backward: psi loads issued back to back (a 1024-thread workgroup runs four wavefronts per
// SIMD and keeps 16 in flight; smaller ones run six, with registers for 8)
template <int WG>
constexpr int kPsiLoads = WG >= 1024 ? 16 : 8;

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, int k) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, k);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int k) {
    const uint32_t lo = readlane_u32((uint32_t)x, k), hi = readlane_u32((uint32_t)(x >> 32), k);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const unsigned lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}
// a team's control words after a team barrier: the barrier orders them, the load only has
// to be coherent (an acquire load would also invalidate the L2)
template <class T>
__device__ __forceinline__ T ld_team(T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_rel(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// per-vertex masks of one team: {seen, nxt} in one 16-byte record
struct Masks {
    uint64_t* p;
    __device__ __forceinline__ uint64_t& seen(uint32_t v) const { return p[2 * (size_t)v]; }
    __device__ __forceinline__ uint64_t& nxt(uint32_t v) const { return p[2 * (size_t)v + 1]; }
    __device__ __forceinline__ ulonglong2 both(uint32_t v) const { return reinterpret_cast<const ulonglong2*>(p)[v]; }
    __device__ __forceinline__ void clear(uint32_t v) const {
        reinterpret_cast<ulonglong2*>(p)[v] = make_ulonglong2(0ull, 0ull);
    }
};

template <int WG>
struct MsbLds {
    uint32_t wsum[WG / 64];
    uint32_t off[WG];       // unit offsets of the chunk's entries
    uint16_t own[2 * WG];   // unit -> chunk entry, for the chunk's first 2 WG units
    uint32_t ev[WG];        // entry vertex
    uint64_t em[WG];        // entry source mask
    uint32_t eb[WG];        // first out-edge
    uint32_t ed[WG];        // out-degree
    int32_t eh[WG];         // accumulator row of a split entry, -1 otherwise
    uint32_t hub_ent[WG];   // accumulator row -> chunk entry
    double hl[WG / 8][64];  // the first accumulator rows (LDS atomics: no wait on memory)
    unsigned long long ws[WG / 64][6];   // per wavefront: reached pairs, examined, entries, visits, pulled
                                         // in-edges, DAG (edge, source) pairs of pulled levels
    uint32_t nhub;
    uint32_t chunk;
    uint32_t ucnt;          // next unit of the chunk to claim
    uint32_t ok;            // 0 once the team gave up on a barrier
    uint64_t ovf;           // sources flagged by this workgroup, flushed to the team at level ends
};

// Team-wide barrier over the workgroups of one team, with a bounded wait.  Makes every
// member's global writes visible to every member.  Returns false if the team has given up.
// Each workgroup first gathers its own writes with a workgroup-scope barrier; only thread 0
// then synchronises at agent scope (one L2 write-back on arrival, one invalidate after the
// wait; the wait itself polls with plain coherent loads).  A team of one workgroup needs
// workgroup scope only.
template <int WG>
__device__ bool team_sync(MsbLds<WG>& L, TeamCtl* c, uint32_t W, CallStats* stats, uint64_t wait_ticks) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        if (W > 1) {
            const uint32_t gen = ld_team(&c->bar_gen);
            // acquire-release: publishes this workgroup's writes, and the last arriver takes
            // every member's before it opens the barrier
            const uint32_t arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == W - 1) {
                __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint64_t t0 = wall_clock64();
                while (ld_team(&c->bar_gen) == gen) {
                    if (ld_team(&c->abort) || wall_clock64() - t0 > wait_ticks) {
                        st_rel(&c->abort, 1u);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            if (ld_team(&c->abort)) ok = 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (!ok) atomicOr(&stats->aborted, 1u);
        L.ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return L.ok != 0u;
}

template <int WG>
__device__ __forceinline__ uint32_t find_owner(const uint32_t* a, uint32_t p) {
    uint32_t lo = 0, len = WG;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (a[lo + half] <= p) lo += half;
        len -= half;
    }
    return lo;
}

// chunk entry of unit u: one LDS read for the first 2 WG units, a search after them
template <int WG>
__device__ __forceinline__ uint32_t owner_of(const MsbLds<WG>& L, uint32_t u) {
    return u < 2 * WG ? (uint32_t)L.own[u] : find_owner<WG>(L.off, u);
}

// each entry records itself as the owner of its units (those inside the table)
template <int WG>
__device__ __forceinline__ void fill_owners(MsbLds<WG>& L, uint32_t off, uint32_t units) {
    const uint32_t end = min(off + units, 2u * WG);
    for (uint32_t q = off; q < end; ++q) L.own[q] = (uint16_t)threadIdx.x;
}

template <int WG>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, uint32_t* wsum) {
    const unsigned lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
        const uint32_t t = wsum[i];
        if (i < (int)w) before += t;
        all += t;
    }
    __syncthreads();
    total = all;
    return before + incl - x;
}

// Collects a level: every vertex whose next-mask is non-zero becomes an entry (w, mask) of
// the team's level list; the mask is folded into seen and the next-mask cleared.  Each
// thread takes kScanUnroll vertices per pass (loads first), each wavefront one list append.
// With pulls enabled (`cur` non-null) it also publishes each entry's lanes and level in `cur`
// and sums, into `pin`, the in-degrees of the vertices that some lane of the batch has still not
// reached: what pulling the next level would read.
constexpr int kScanUnroll = 8;
__device__ __forceinline__ uint32_t collect_level(const MsbArgs& a, TeamCtl* c, const Masks mk, uint32_t* lv,
                                                  uint64_t* lm, uint32_t first, uint32_t stride, uint32_t n,
                                                  ulonglong2* cur, uint64_t lanes, uint32_t tag, uint32_t& pin) {
    const unsigned lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t sdeg = 0;
    for (uint32_t b0 = first; b0 < n; b0 += stride * kScanUnroll) {
        uint64_t m[kScanUnroll];
        uint64_t bal[kScanUnroll];
        uint32_t cnt = 0;
        if (cur) {
#pragma unroll
            for (int j = 0; j < kScanUnroll; ++j) {
                const uint32_t w = b0 + j * stride;
                m[j] = 0ull;
                if (w < n) {
                    const ulonglong2 q = mk.both(w);
                    m[j] = q.y;
                    if (lanes & ~(q.x | q.y)) pin += a.csc_ptr[w + 1] - a.csc_ptr[w];
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < kScanUnroll; ++j) {
                const uint32_t w = b0 + j * stride;
                m[j] = w < n ? mk.nxt(w) : 0ull;
            }
        }
#pragma unroll
        for (int j = 0; j < kScanUnroll; ++j) {
            bal[j] = __ballot(m[j] != 0ull);
            cnt += (uint32_t)__builtin_popcountll(bal[j]);
        }
        if (!cnt) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&c->tail, cnt);
        base = __shfl(base, 0, 64);
#pragma unroll
        for (int j = 0; j < kScanUnroll; ++j) {
            const uint32_t w = b0 + j * stride;
            if (m[j]) {
                const uint32_t pos = base + (uint32_t)__builtin_popcountll(bal[j] & below);
                lv[pos] = w;
                lm[pos] = m[j];
                __hip_atomic_fetch_or((unsigned long long*)&mk.seen(w), (unsigned long long)m[j], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                mk.nxt(w) = 0ull;
                if (cur) cur[w] = make_ulonglong2(m[j], (unsigned long long)tag);
                sdeg += a.row_ptr[w + 1] - a.row_ptr[w];
            }
            base += (uint32_t)__builtin_popcountll(bal[j]);
        }
    }
    return sdeg;
}

// row updates of one forward unit, lane per source: sig[w][s] += sv for every DAG edge (v, w)
// of the unit and s in its mask; the edges are taken from the ballot in lane order, their
// successor and mask read from that lane's registers.  No value is returned: no wait.
__device__ __forceinline__ void rows_add(uint32_t* sig, uint32_t w, uint64_t dag, uint32_t sv) {
    const unsigned lane = lane_id();
    uint64_t bal = __ballot(dag != 0ull);
    while (bal) {
        const int k = __builtin_ctzll(bal);
        bal &= bal - 1ull;
        const uint32_t wj = readlane_u32(w, k);
        const uint64_t dj = readlane_u64(dag, k);
        if ((dj >> lane) & 1ull)
            __hip_atomic_fetch_add(&sig[(size_t)wj * 64 + lane], sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Forward work of one wavefront: two units, A = out-edges [e0A, e1A) of the level-d entry
// (vA, fA) and B likewise (e0B == e1B: none).  Each unit tests up to 64 edges at once; every
// load of both units is issued before the first dependent use, so their round trips overlap.
template <int WG>
__device__ __forceinline__ void fwd_units(const MsbArgs& a, MsbLds<WG>& L, const Masks mk, uint32_t* sig,
                                          uint32_t vA, uint64_t fA, uint32_t e0A, uint32_t e1A, uint32_t vB,
                                          uint64_t fB, uint32_t e0B, uint32_t e1B) {
    const unsigned lane = lane_id();
    const uint32_t eA = e0A + lane, eB = e0B + lane;
    const bool okA = eA < e1A, okB = eB < e1B;
    const bool actA = (fA >> lane) & 1ull, actB = (fB >> lane) & 1ull;
    // Every load is issued by every lane, idle lanes repeating an address of an active lane
    // (no extra sectors): loads without branches around them keep the wait counts exact, so
    // the second unit's gathers do not wait for the first unit's.  An empty unit B (fB = 0,
    // e0B = e1B) reads vertex 0's row and edge 0, which exist whenever a unit does.
    const uint32_t lA = actA ? lane : (uint32_t)__builtin_ctzll(fA | (1ull << 63));
    const uint32_t lB = actB ? lane : (uint32_t)__builtin_ctzll(fB | (1ull << 63));
    const uint32_t sA = sig[(size_t)vA * 64 + lA];
    const uint32_t sB = sig[(size_t)vB * 64 + lB];
    const uint32_t wA0 = a.col[okA ? eA : e1A - 1];
    const uint32_t wB0 = a.col[okB ? eB : (e1B > e0B ? e1B - 1 : 0u)];
    __builtin_amdgcn_sched_barrier(0);   // the four independent loads above go out first
    const uint32_t wA = okA ? wA0 : vA, wB = okB ? wB0 : vB;   // valid vertex ids only
    const ulonglong2 qA = mk.both(wA);
    const ulonglong2 qB = mk.both(wB);
    const uint32_t svA = actA ? sA : 0u, svB = actB ? sB : 0u;
    const uint64_t dagA = okA ? (fA & ~qA.x) : 0ull, dagB = okB ? (fB & ~qB.x) : 0ull;
    // bits only get set during a level, so a plain read that already shows every bit of dag
    // (stale reads show fewer) proves the OR would change nothing: skip it
    if ((dagA & ~qA.y) != 0ull)
        __hip_atomic_fetch_or((unsigned long long*)&mk.nxt(wA), (unsigned long long)dagA, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    if ((dagB & ~qB.y) != 0ull)
        __hip_atomic_fetch_or((unsigned long long*)&mk.nxt(wB), (unsigned long long)dagB, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    // a source whose count here could carry its successors' sums past 32 bits is handed on
    const uint64_t risk = __ballot(svA > a.sig_cap || svB > a.sig_cap);
    if (lane == 0 && risk) atomicOr((unsigned long long*)&L.ovf, (unsigned long long)risk);
    rows_add(sig, wA, dagA, svA);
    rows_add(sig, wB, dagB, svB);
}

// One unit of a pulled level: in-edges [e0, e1) of vertex w, whose lanes `un` are unreached.
// Lane per in-edge first (in-neighbour x and its level-d lanes), then lane per source: the
// counts of the in-neighbours holding the lane are summed, kPullLoads rows in flight.  A vertex
// with more in-edges than one unit (`split`) adds its partial sums and next-mask with atomics;
// otherwise it is the only writer of its row and next-mask.  Counts this lane's in-edge read and
// its DAG (edge, source) pairs into `read` and `pairs`.
constexpr int kPullLoads = 16;
template <int WG>
__device__ __forceinline__ void pull_unit(const MsbArgs& a, MsbLds<WG>& L, const Masks mk, uint32_t* sig,
                                              const ulonglong2* cur, uint32_t w, uint64_t un, uint32_t e0,
                                              uint32_t e1, bool split, uint64_t tag, uint32_t& read,
                                              uint32_t& pairs) {
    const unsigned lane = lane_id();
    const uint32_t e = e0 + lane;
    const bool ok = e < e1;
    const uint32_t x = a.csc_row[ok ? e : e1 - 1];
    const ulonglong2 c = cur[x];
    const uint64_t lx = (ok && c.y == tag) ? (c.x & un) : 0ull;   // lanes with x on level d: (x, w) on their DAG
    uint64_t rem = __ballot(lx != 0ull);
    uint64_t nx = 0;
    uint32_t acc = 0;
    bool risk = false;
    while (rem) {
        uint32_t y[kPullLoads];
#pragma unroll
        for (int q = 0; q < kPullLoads; ++q) {
            y[q] = 0u;
            if (rem) {
                const int k = __builtin_ctzll(rem);
                rem &= rem - 1ull;
                const uint32_t xk = readlane_u32(x, k);
                const uint64_t mk_ = readlane_u64(lx, k);
                nx |= mk_;
                if ((mk_ >> lane) & 1ull) y[q] = sig[(size_t)xk * 64 + lane];
            }
        }
#pragma unroll
        for (int q = 0; q < kPullLoads; ++q) {
            risk |= y[q] > a.sig_cap;
            acc += y[q];
        }
    }
    if (nx) {
        const bool mine = (nx >> lane) & 1ull;
        if (!split) {
            if (lane == 0) mk.nxt(w) = nx;
            if (mine) sig[(size_t)w * 64 + lane] = acc;
        } else {
            if (lane == 0)
                __hip_atomic_fetch_or((unsigned long long*)&mk.nxt(w), (unsigned long long)nx, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            if (mine && acc)
                __hip_atomic_fetch_add(&sig[(size_t)w * 64 + lane], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // a lane that summed a count beyond the cap is handed on, as in the pushed levels
    const uint64_t flag = __ballot(risk);
    if (lane == 0 && flag) atomicOr((unsigned long long*)&L.ovf, (unsigned long long)flag);
    read += ok ? 1u : 0u;
    pairs += (uint32_t)__builtin_popcountll(lx);
}

// finishes list entry idx = (v, f) of level d with the summed successor psi in `acc`;
// `count` is this lane's sigma_s(v), read by the caller
__device__ __forceinline__ void finish_entry(uint32_t* sig, double* psi, double* bcp, uint32_t idx, uint32_t v,
                                             uint64_t f, double acc, uint32_t count, uint32_t my_src,
                                             uint32_t deg, unsigned long long* ws) {
    const unsigned lane = lane_id();
    double c = 0.0;
    if ((f >> lane) & 1ull) {
        const double sigma = (double)count;
        const double delta = sigma * acc;
        psi[(size_t)v * 64 + lane] = (1.0 + delta) / sigma;
        sig[(size_t)v * 64 + lane] = 0u;   // the count's last use: cleared for the next batch
        if (my_src != v) c = delta;
    }
    c = wave_sum(c);
    if (lane == 0) {
        bcp[idx] = c;   // added to BC[v] when the batch is reset: no atomic in the sweep
        const uint32_t pc = (uint32_t)__builtin_popcountll(f);
        atomicAdd(&ws[0], (unsigned long long)pc);   // this wavefront's counters, in LDS
        atomicAdd(&ws[1], (unsigned long long)pc * deg);
        atomicAdd(&ws[2], 1ull);
        atomicAdd(&ws[3], (unsigned long long)deg);
    }
}

// Claims `k` consecutive units of the current chunk for this wavefront (units vary in cost, so
// wavefronts take them as they finish rather than in a fixed round-robin)
template <int WG>
__device__ __forceinline__ uint32_t claim_units(MsbLds<WG>& L, uint32_t k) {
    uint32_t u = 0;
    if (lane_id() == 0) u = atomicAdd(&L.ucnt, k);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)u);
}

// Claims the next chunk of the current phase for this workgroup (team-wide counter).
template <int WG>
__device__ __forceinline__ uint32_t claim_chunk(MsbLds<WG>& L, TeamCtl* c) {
    if (threadIdx.x == 0) {
        L.chunk = atomicAdd(&c->cc, 1u);
        L.ucnt = 0;   // every wavefront left the previous chunk's unit loop at its last barrier
    }
    __syncthreads();
    const uint32_t ch = L.chunk;
    __syncthreads();
    return ch;
}

// Workgroups of up to 512 threads are built for six wavefronts per SIMD (80 VGPRs; the
// loop-invariant state pointers spill): three 512-thread workgroups fill a compute unit's LDS,
// and the extra wavefronts hide more of the gather latency (R-MAT scale 20: 27.8 -> 26.1 ms)
template <int WG>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WG <= 512 ? 6 : 1)))
k_msb(MsbArgs a) {
    __shared__ MsbLds<WG> L;
    const unsigned tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    constexpr unsigned NW = WG / 64;
    const uint32_t total = *a.plan_count;
    const uint32_t nbatch = (total + 63) / 64;
    // Team size, chosen on the device from the batch count: the grid is split into at most
    // min(batches, pool slots) teams, each at most one XCD's share of the grid.  With 8-way
    // round-robin dispatch, workgroups b, b+8, b+16, ... share an XCD; when W divides that
    // stride group, a team is W of them, so its batch state stays behind one L2.
    const uint32_t want = max(1u, min(nbatch, a.pool_teams));
    const uint32_t per_xcd = gridDim.x / 8;
    uint32_t W = a.team_size ? a.team_size : max(1u, min(max(per_xcd, 1u), gridDim.x / want));
    W = min(W, gridDim.x);
    uint32_t team, member;
    if (gridDim.x % 8 == 0) {
        // XCD-major numbering: a team takes consecutive workgroups of one XCD and spills into
        // the next only when W does not divide the per-XCD count (a team of 28 out of 32 per
        // XCD spans at most two L2s instead of all eight)
        const uint32_t lin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
        team = lin / W;
        member = lin % W;
    } else {
        team = blockIdx.x / W;
        member = blockIdx.x % W;
    }
    if (team >= a.pool_teams || team >= (gridDim.x / W)) return;   // no state slot for this workgroup
    const bool leader = member == 0;
    TeamCtl* ctl = a.ctl + team;
    const size_t n = (size_t)a.n;
    const Masks mk{a.masks + (size_t)team * a.mask_stride};
    uint32_t* sig = a.sig + (size_t)team * a.sig_stride;
    double* psi = a.psi + (size_t)team * a.psi_stride;
    uint64_t* bnx = a.bnx + (size_t)team * a.bnx_stride;
    ulonglong2* cur = a.pull16 ? a.cur + (size_t)team * a.cur_stride : nullptr;
    uint32_t pull_levels = 0;   // leader's thread 0: levels pulled, and the out-edges they did not push
    uint64_t pull_skip = 0;
    double* hacc = a.hacc + (size_t)blockIdx.x * a.hub_rows * 64;
    double* bcp = a.bcp + (size_t)team * a.cap;
    constexpr uint32_t HL = WG / 8;   // accumulator rows in LDS
    uint32_t* lv = a.lst_v + (size_t)team * a.cap;
    uint64_t* lm = a.lst_m + (size_t)team * a.cap;
    uint32_t* lvl = a.lvl + (size_t)team * (a.max_levels + 2);
    const uint32_t gtid = member * WG + tid, gthreads = W * WG;
    // entries per chunk: WG / clamp(W, 2, 8).  Larger teams take smaller chunks, so the last
    // chunks of a level (and chunks holding hubs) keep fewer members waiting at the level's
    // barrier; R-MAT scale 20 (W = 16) ran 358 GTEPS with whole-WG chunks, 460 with WG/8
    const uint32_t CH = WG / min(8u, max(2u, W));
    const uint32_t gwave = member * NW + wave, gwaves = W * NW;
    uint32_t dagc = 0;
    uint32_t n_done = 0, levels_max = 0, scans = 0;
    uint64_t cyc[3] = {0, 0, 0};   // thread 0: clock cycles in forward, backward, reset

    if (lane == 0)
        for (int q = 0; q < 6; ++q) L.ws[wave][q] = 0ull;
    if (tid == 0) {
        L.nhub = 0;
        L.ovf = 0;
    }
    for (;;) {
        if (leader && tid == 0) {
            ctl->batch = atomicAdd(&a.stats->work_head, 1u);
            ctl->tail = 0;
            ctl->cc = 0;
            ctl->ovf = 0;
            ctl->sdeg[0] = ctl->sdeg[1] = 0;
            ctl->pin[0] = ctl->pin[1] = 0;
        }
        if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) break;
        const uint32_t b = ld_team(&ctl->batch);
        if (b >= nbatch) break;
        const uint32_t base = b * 64;
        const uint32_t nl = min(64u, total - base);
        const uint64_t lanes = nl == 64 ? ~0ull : ((1ull << nl) - 1ull);
        const uint32_t my_src = lane < nl ? a.plan[base + lane] : 0xffffffffu;
        if (leader && wave == 0 && lane < nl) {   // level 0: the sources themselves
            __hip_atomic_fetch_or((unsigned long long*)&mk.nxt(my_src), (unsigned long long)(1ull << lane),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sig[(size_t)my_src * 64 + lane] = 1u;
        }
        // ---------------- forward sweep ----------------
        uint64_t t_phase = clock64();
        uint32_t lo = 0, d = 0;
        bool stopped = false;       // every thread takes the same decision from the same values
        bool aborted = false;
        for (;;) {
            if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) {
                aborted = true;
                break;
            }
            if (leader && tid == 0) {
                ctl->cc = 0;                       // chunk counter of this level's expansion
                ctl->sdeg[(d + 1) & 1] = 0;        // filled by the next level's scan
                ctl->pin[(d + 1) & 1] = 0;
            }
            // level d: the vertices some source reached in the previous expansion
            uint32_t pin = 0;
            uint32_t sdeg = collect_level(a, ctl, mk, lv, lm, member * WG + tid, gthreads, (uint32_t)n, cur, lanes,
                                          d + 1, pin);
            sdeg = wave_sum_u32(sdeg);
            if (lane == 0 && sdeg) atomicAdd(&ctl->sdeg[d & 1], sdeg);
            if (cur) {
                pin = wave_sum_u32(pin);
                if (lane == 0 && pin) atomicAdd(&ctl->pin[d & 1], pin);
            }
            if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) {
                aborted = true;
                break;
            }
            const uint32_t hi = ld_team(&ctl->tail);
            if (leader && tid == 0) {
                lvl[d] = lo;
                lvl[d + 1] = hi;
            }
            if (hi == lo) break;   // level d is empty: the sweep is over (levels 0..d-1)
            const uint64_t room = (uint64_t)a.cap - hi;
            const uint32_t lsdeg = ld_team(&ctl->sdeg[d & 1]);
            if (d + 2 > a.max_levels || room < min<uint64_t>(n, lsdeg)) {
                stopped = true;
                d += 1;
                break;
            }
            // the same values in every member: the whole team takes the same direction
            const bool pull = cur && (uint64_t)ld_team(&ctl->pin[d & 1]) * 16u < (uint64_t)lsdeg * a.pull16;
            if (pull && leader && tid == 0) {
                ++pull_levels;
                pull_skip += lsdeg;
            }
            for (;;) {   // pulled level: chunks of WG vertices, units of <= 64 in-edges
                if (!pull) break;
                const uint32_t ch = claim_chunk(L, ctl);
                const uint32_t c0 = ch * WG;
                if (c0 >= (uint32_t)n) break;
                const uint32_t w = c0 + tid;
                uint32_t beg = 0, deg = 0;
                uint64_t un = 0;
                if (w < (uint32_t)n) {
                    un = lanes & ~mk.seen(w);
                    if (un) {
                        beg = a.csc_ptr[w];
                        deg = a.csc_ptr[w + 1] - beg;
                    }
                }
                uint32_t units;
                const uint32_t off = block_excl_scan<WG>((deg + 63) / 64, units, L.wsum);
                L.off[tid] = off;
                fill_owners<WG>(L, off, (deg + 63) / 64);
                L.ev[tid] = w;
                L.em[tid] = un;
                L.eb[tid] = beg;
                L.ed[tid] = deg;
                __syncthreads();
                uint32_t read = 0, pairs = 0;
                for (;;) {
                    const uint32_t u = claim_units(L, 1u);
                    if (u >= units) break;
                    const uint32_t j = owner_of<WG>(L, u);
                    const uint32_t e0 = L.eb[j] + (u - L.off[j]) * 64;
                    const uint32_t e1 = min(L.eb[j] + L.ed[j], e0 + 64);
                    pull_unit<WG>(a, L, mk, sig, cur, L.ev[j], L.em[j], e0, e1, L.ed[j] > 64, d + 1, read, pairs);
                }
                read = wave_sum_u32(read);
                pairs = wave_sum_u32(pairs);
                if (lane == 0 && read) atomicAdd(&L.ws[wave][4], (unsigned long long)read);
                if (lane == 0 && pairs) atomicAdd(&L.ws[wave][5], (unsigned long long)pairs);
                __syncthreads();
            }
            for (;;) {   // pushed level
                if (pull) break;
                const uint32_t ch = claim_chunk(L, ctl);
                const uint32_t c0 = lo + ch * CH;
                if (c0 >= hi) break;
                const uint32_t i = c0 + tid;
                uint32_t v = 0, beg = 0, deg = 0;
                uint64_t f = 0;
                if (tid < CH && i < hi) {
                    v = lv[i];
                    f = lm[i];
                    beg = a.row_ptr[v];
                    deg = a.row_ptr[v + 1] - beg;
                }
                uint32_t units;
                const uint32_t off = block_excl_scan<WG>((deg + 63) / 64, units, L.wsum);
                L.off[tid] = off;
                fill_owners<WG>(L, off, (deg + 63) / 64);
                L.ev[tid] = v;
                L.em[tid] = f;
                L.eb[tid] = beg;
                L.ed[tid] = deg;
                __syncthreads();
                for (;;) {   // units u and u + 1
                    const uint32_t u = claim_units(L, 2u);
                    if (u >= units) break;
                    const uint32_t j = owner_of<WG>(L, u);
                    const uint32_t e0 = L.eb[j] + (u - L.off[j]) * 64;
                    const uint32_t e1 = min(L.eb[j] + L.ed[j], e0 + 64);
                    const uint32_t u2 = u + 1;
                    uint32_t v2 = 0, e02 = 0, e12 = 0;
                    uint64_t f2 = 0;
                    if (u2 < units) {
                        const uint32_t j2 = owner_of<WG>(L, u2);
                        v2 = L.ev[j2];
                        f2 = L.em[j2];
                        e02 = L.eb[j2] + (u2 - L.off[j2]) * 64;
                        e12 = min(L.eb[j2] + L.ed[j2], e02 + 64);
                    }
                    fwd_units<WG>(a, L, mk, sig, L.ev[j], L.em[j], e0, e1, v2, f2, e02, e12);
                }
                __syncthreads();
            }
            if (tid == 0) {   // flush this workgroup's level results to the team
                if (L.ovf) atomicOr((unsigned long long*)&ctl->ovf, (unsigned long long)L.ovf);
                L.ovf = 0;
            }
            lo = hi;
            ++d;
        }
        if (aborted) break;
        {
            const uint64_t t = clock64();
            cyc[0] += t - t_phase;
            t_phase = t;
        }
        const uint32_t nlev = d;            // levels 0..nlev-1 hold entries
        const uint32_t n_entries = ld_team(&ctl->tail);
        const uint64_t ovf = stopped ? lanes : (ld_team(&ctl->ovf) & lanes);
        // ---------------- backward sweep ----------------
        if (!stopped) {
            if (leader && tid == 0) lvl[nlev + 1] = lvl[nlev];
            for (int dd = (int)nlev - 1; dd >= 0 && !aborted; --dd) {
                if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) {
                    aborted = true;
                    break;
                }
                const uint32_t lo_d = lvl[dd], hi_d = lvl[dd + 1];
                const uint32_t lo_n = lvl[dd + 1], hi_n = lvl[dd + 2];
                if (leader && tid == 0) ctl->cc = 0;
                for (uint32_t i = lo_n + gtid; i < hi_n; i += gthreads) bnx[lv[i]] = lm[i] & ~ovf;
                if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) {
                    aborted = true;
                    break;
                }
                for (;;) {
                    const uint32_t ch = claim_chunk(L, ctl);
                    const uint32_t c0 = lo_d + ch * CH;
                    if (c0 >= hi_d) break;
                    const uint32_t i = c0 + tid;
                    uint32_t v = 0, beg = 0, deg = 0, np = 0;
                    uint64_t f = 0;
                    if (tid < CH && i < hi_d) {
                        v = lv[i];
                        f = lm[i] & ~ovf;
                        beg = a.row_ptr[v];
                        deg = a.row_ptr[v + 1] - beg;
                        if (f) np = deg > 64 ? (deg + 63) / 64 : 1u;
                    }
                    int32_t row = -1;
                    if (np > 1) {
                        row = (int32_t)atomicAdd(&L.nhub, 1u);
                        L.hub_ent[row] = tid;
                        if ((uint32_t)row < HL) {
                            for (int q = 0; q < 64; ++q) L.hl[row][q] = 0.0;
                        } else {
                            for (int q = 0; q < 64; ++q) hacc[(size_t)(row - HL) * 64 + q] = 0.0;
                        }
                    }
                    uint32_t units;
                    const uint32_t off = block_excl_scan<WG>(np, units, L.wsum);
                    L.off[tid] = off;
                    fill_owners<WG>(L, off, np);
                    L.ev[tid] = v;
                    L.em[tid] = f;
                    L.eb[tid] = beg;
                    L.ed[tid] = deg;
                    L.eh[tid] = row;
                    // the accumulator rows belong to this workgroup alone: workgroup scope
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __syncthreads();
                    for (;;) {
                        const uint32_t u = claim_units(L, 1u);
                        if (u >= units) break;
                        const uint32_t j = owner_of<WG>(L, u);
                        const uint32_t vj = L.ev[j];
                        const uint64_t fj = L.em[j];
                        const uint32_t dj = L.ed[j];
                        const uint32_t e0 = L.eb[j] + (u - L.off[j]) * 64;
                        const uint32_t e1 = min(L.eb[j] + dj, e0 + 64);
                        const uint32_t e = e0 + lane;
                        const int32_t hr = L.eh[j];
                        // the entry's own counts, read early when this unit finishes the entry
                        const uint32_t cnt_v = (hr < 0 && ((fj >> lane) & 1ull)) ? sig[(size_t)vj * 64 + lane] : 0u;
                        uint32_t w = 0;
                        uint64_t sm = 0;
                        if (e < e1) {
                            w = a.col[e];
                            sm = fj & bnx[w];
                        }
                        dagc += (uint32_t)__builtin_popcountll(sm);
                        // lane per source: sum psi over the unit's successors, taken from the
                        // ballot kPsiLoads<WG> at a time so that as many loads are in flight
                        uint64_t rem = __ballot(sm != 0ull);
                        double acc = 0.0;
                        while (rem) {
                            double x[kPsiLoads<WG>];
#pragma unroll
                            for (int t = 0; t < kPsiLoads<WG>; ++t) {
                                x[t] = 0.0;
                                if (rem) {
                                    const int k = __builtin_ctzll(rem);
                                    rem &= rem - 1ull;
                                    const uint32_t wt = readlane_u32(w, k);
                                    const uint64_t mt = readlane_u64(sm, k);
                                    if ((mt >> lane) & 1ull) x[t] = psi[(size_t)wt * 64 + lane];
                                }
                            }
#pragma unroll
                            for (int t = 0; t < kPsiLoads<WG>; ++t) acc += x[t];
                        }
                        if (hr < 0) {
                            finish_entry(sig, psi, bcp, c0 + j, vj, fj, acc, cnt_v, my_src, dj, L.ws[wave]);
                        } else if (((fj >> lane) & 1ull) && acc != 0.0) {
                            if ((uint32_t)hr < HL)
                                unsafeAtomicAdd(&L.hl[hr][lane], acc);
                            else
                                unsafeAtomicAdd(&hacc[(size_t)(hr - HL) * 64 + lane], acc);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __syncthreads();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    const uint32_t nh = L.nhub;
                    for (uint32_t h = wave; h < nh; h += NW) {
                        const uint32_t j = L.hub_ent[h];
                        const uint32_t vj = L.ev[j];
                        const uint64_t fj = L.em[j];
                        const uint32_t cnt_v = ((fj >> lane) & 1ull) ? sig[(size_t)vj * 64 + lane] : 0u;
                        const double acc = h < HL ? L.hl[h][lane] : hacc[(size_t)(h - HL) * 64 + lane];
                        finish_entry(sig, psi, bcp, c0 + j, vj, fj, acc, cnt_v, my_src, L.ed[j], L.ws[wave]);
                    }
                    __syncthreads();
                    if (tid == 0) L.nhub = 0;
                    __syncthreads();
                }
                // no clearing pass: a stale mask left in bnx[w] by a deeper level L >= d + 2
                // never meets an entry of level d with an edge to w (such a source would
                // reach w within d + 1), and the reset clears every listed vertex's masks
            }
        }
        if (aborted) break;
        {
            const uint64_t t = clock64();
            cyc[1] += t - t_phase;
            t_phase = t;
        }
        // ---------------- reset the touched state ----------------
        if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) break;
        // entries, thread per entry: mask records, and the BC contributions of finished entries
        for (uint32_t i = gtid; i < n_entries; i += gthreads) {
            const uint32_t v = lv[i];
            const uint64_t m = lm[i];
            mk.clear(v);
            bnx[v] = 0ull;
            if (cur) cur[v] = make_ulonglong2(0ull, 0ull);
            if (!stopped && (m & ~ovf)) {
                const double c = bcp[i];
                if (c != 0.0) unsafeAtomicAdd(&a.bc[a.iperm ? a.iperm[v] : v], c);
            }
        }
        // counts, lane per source: the backward sweep cleared those of finished entries; what
        // remains are the flagged sources' (psi is written before it is read)
        const uint64_t left = stopped ? ~0ull : ovf;
        if (left)
            for (uint32_t i = gwave; i < n_entries; i += gwaves) {
                const uint32_t v = lv[i];
                const uint64_t m = lm[i] & left;
                if ((m >> lane) & 1ull) sig[(size_t)v * 64 + lane] = 0u;
            }
        // sources this kernel did not finish go to the per-source kernel
        if (leader && tid == 0) {
            if (ovf) {
                const uint32_t cnt = (uint32_t)__builtin_popcountll(ovf);
                uint32_t pos = atomicAdd(a.retry_count, cnt);
                atomicAdd(&a.stats->handoffs, cnt);
                uint64_t m = ovf;
                while (m) {
                    const int s = __builtin_ctzll(m);
                    m &= m - 1ull;
                    a.retry[pos++] = a.plan[base + s];
                }
            }
            n_done += (uint32_t)__builtin_popcountll(lanes & ~ovf);
            if (!stopped) levels_max = max(levels_max, nlev);
            scans += stopped ? nlev : nlev + 1;   // the last pass found the empty level
        }
        if (!team_sync(L, ctl, W, a.stats, a.wait_ticks)) break;
        cyc[2] += clock64() - t_phase;
    }
    // counters of everything this workgroup finished
    const uint32_t g_w = wave_sum_u32(dagc);
    if (lane == 0) {
        const unsigned long long r_w = L.ws[wave][0], e_w = L.ws[wave][1], n_w = L.ws[wave][2], v_w = L.ws[wave][3];
        if (r_w) atomicAdd((unsigned long long*)&a.stats->reached, r_w);
        if (e_w) atomicAdd((unsigned long long*)&a.stats->examined, e_w);
        if (g_w) atomicAdd((unsigned long long*)&a.stats->dag_edges, (unsigned long long)g_w);
        if (n_w) atomicAdd((unsigned long long*)&a.stats->entries, n_w);
        if (v_w) atomicAdd((unsigned long long*)&a.stats->edge_visits, v_w);
        const unsigned long long p_w = L.ws[wave][4], q_w = L.ws[wave][5];
        if (p_w) atomicAdd((unsigned long long*)&a.stats->pull_edges, p_w);
        if (q_w) atomicAdd((unsigned long long*)&a.stats->pull_pairs, q_w);
    }
    if (tid == 0) {
        if (n_done) atomicAdd(&a.stats->n_done, n_done);
        if (scans) atomicAdd((unsigned long long*)&a.stats->scans, (unsigned long long)scans);
        if (levels_max) atomicMax(&a.stats->levels_max, levels_max);
        if (pull_levels) atomicAdd((unsigned long long*)&a.stats->pull_levels, (unsigned long long)pull_levels);
        if (pull_skip) atomicAdd((unsigned long long*)&a.stats->pull_skip, (unsigned long long)pull_skip);
        for (int i = 0; i < 3; ++i)
            if (cyc[i]) atomicAdd((unsigned long long*)&a.stats->cycles[i], (unsigned long long)cyc[i]);
    }
}

// ---- source plan: valid sources with out-edges, in the graph's batching order ----
// All vertices as sources: the plan is the order itself (its vertices with out-edges come
// first).  A source list is counting-sorted by rank into kPlanBuckets buckets of consecutive
// ranks (exact order for graphs of up to kPlanBuckets vertices).
constexpr uint32_t kPlanBuckets = 65536;

__device__ __forceinline__ uint32_t plan_bucket(const uint32_t* rank, uint32_t s, uint32_t n, uint32_t nb) {
    const uint32_t r = rank ? rank[s] : s;
    return (uint32_t)(((uint64_t)r * nb) / n);
}

__global__ void k_plan_all(const uint32_t* order, uint32_t n, uint32_t active, const uint32_t* perm, uint32_t* plan,
                           uint32_t* plan_count, CallStats* stats) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < active; i += gridDim.x * blockDim.x) {
        const uint32_t s = order ? order[i] : i;
        plan[i] = perm ? perm[s] : s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        plan_count[0] = active;
        // sources without out-edges: finished here (they reach only themselves)
        const uint32_t idle = n - active;
        stats->n_done += idle;
        stats->reached += idle;
        if (idle && stats->levels_max < 1) stats->levels_max = 1;
    }
}

// hist[0..nb): sources per bucket; hist[nb]: sources without out-edges
__global__ void k_plan_hist(const uint32_t* row_ptr, const uint32_t* rank, const uint32_t* srcs, uint32_t k,
                            uint32_t n, uint32_t nb, uint32_t* hist, CallStats* stats) {
    uint32_t bad = 0, idle = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t s = srcs ? srcs[i] : i;
        if (s >= n) {
            ++bad;
        } else if (row_ptr[s + 1] == row_ptr[s]) {
            ++idle;
        } else {
            atomicAdd(&hist[plan_bucket(rank, s, n, nb)], 1u);
        }
    }
    if (bad) atomicAdd(&stats->bad_source, bad);
    if (idle) atomicAdd(&hist[nb], idle);
}

// one workgroup of 1024 threads: exclusive scan of hist[0..nb) in place
__global__ void __launch_bounds__(1024) k_plan_scan(uint32_t* hist, uint32_t nb, uint32_t* plan_count,
                                                    CallStats* stats) {
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x, per = (nb + 1023) / 1024;
    const uint32_t b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    for (uint32_t i = b0; i < b1; ++i) sum += hist[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {   // inclusive Hillis-Steele scan of the parts
        const uint32_t y = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (uint32_t i = b0; i < b1; ++i) {
        const uint32_t c = hist[i];
        hist[i] = run;
        run += c;
    }
    if (t == 1023) {
        plan_count[0] = part[1023];
        const uint32_t idle = hist[nb];
        stats->n_done += idle;
        stats->reached += idle;
        if (idle && stats->levels_max < 1) stats->levels_max = 1;
    }
}

__global__ void k_plan_scatter(const uint32_t* row_ptr, const uint32_t* rank, const uint32_t* srcs, uint32_t k,
                               uint32_t n, uint32_t nb, const uint32_t* perm, uint32_t* cursor, uint32_t* plan) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t s = srcs ? srcs[i] : i;
        if (s >= n || row_ptr[s + 1] == row_ptr[s]) continue;
        plan[atomicAdd(&cursor[plan_bucket(rank, s, n, nb)], 1u)] = perm ? perm[s] : s;
    }
}

__global__ void k_zero_u32(uint32_t* p, uint32_t count) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_zero_u64(uint64_t* p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

const void* msb_fn(int wg) {
    switch (wg) {
        case 256: return (const void*)k_msb<256>;
        case 512: return (const void*)k_msb<512>;
        default: return (const void*)k_msb<1024>;
    }
}

}  // namespace

int msb_norm_wg(int wg) { return wg <= 256 ? 256 : (wg <= 512 ? 512 : 1024); }

int msb_occupancy(int wg) {
    int per_cu = 0;
    BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, msb_fn(wg), wg, 0));
    return per_cu;
}

// Device state of the batched path for one graph size, reused between calls.
// Team arrays are staggered by an odd number of 4 KiB pages so that the same vertex of
// different teams does not map to the same memory channel.
constexpr uint64_t kStaggerWords = 37 * 512;

struct MsbPool {
    int teams = 0, wgs = 0;
    uint32_t n = 0, cap = 0, max_levels = 0, hub_rows = 0;
    uint64_t mask_stride = 0, sig_stride = 0, psi_stride = 0, bnx_stride = 0;
    TeamCtl* ctl = nullptr;
    uint64_t *masks = nullptr, *lst_m = nullptr, *bnx = nullptr;
    ulonglong2* cur = nullptr;
    uint64_t cur_stride = 0;
    uint32_t* sig = nullptr;
    double *psi = nullptr, *bcp = nullptr;
    double* hacc = nullptr;
    uint32_t *lst_v = nullptr, *lvl = nullptr;
    uint32_t* plan = nullptr;       // [plan_cap]
    uint32_t* retry = nullptr;      // [plan_cap]
    uint32_t plan_cap = 0;
    uint32_t* small = nullptr;      // [80] plan_count, [81] retry_count
    uint32_t* bhist = nullptr;      // [kPlanBuckets + 1] plan histogram / cursors
    int device = -1;                // where the arrays live, and their size in bytes
    size_t bytes = 0;
};

// Bytes held by the batched pools of every graph handle, per device.  A handle keeps its pool
// between calls, so without a shared bound many large handles would each take half of what
// the others left.
static std::atomic<size_t> g_pool_bytes[64];

size_t msb_team_bytes(uint32_t n, uint32_t cap, uint32_t max_levels) {
    return sizeof(TeamCtl) + (size_t)n * (16 + 8 + 16 + 256 + 512) + 5 * kStaggerWords * 8 + (size_t)cap * 20 +
           4 * ((size_t)max_levels + 2);
}

void msb_pool_free(MsbPool& p) {
    for (void* q : {(void*)p.ctl, (void*)p.masks, (void*)p.bnx, (void*)p.cur, (void*)p.sig, (void*)p.psi, (void*)p.bcp, (void*)p.lst_m, (void*)p.hacc,
                    (void*)p.lst_v, (void*)p.lvl, (void*)p.plan, (void*)p.retry, (void*)p.small, (void*)p.bhist})
        if (q) (void)hipFree(q);
    if (p.device >= 0 && p.device < 64) g_pool_bytes[p.device] -= p.bytes;
    p = MsbPool{};
}

MsbPool* msb_pool_new() { return new MsbPool(); }
void msb_pool_delete(MsbPool* p) {
    if (p) {
        msb_pool_free(*p);
        delete p;
    }
}
// A team that gave up on a barrier leaves its state dirty: drop the pool.
void msb_pool_discard(MsbPool* p) {
    if (p) msb_pool_free(*p);
}

static void msb_pool_ensure(MsbPool& p, int device, uint32_t n, int teams, int wgs, uint32_t cap,
                            uint32_t max_levels, uint32_t hub_rows, uint32_t plan_cap, hipStream_t st) {
    // a pool built for a larger graph serves a smaller one: its arrays are all zero between
    // batches, and the kernel takes its strides from the pool
    if (p.masks && p.n >= n && p.teams >= teams && p.wgs >= wgs && p.cap >= cap && p.max_levels >= max_levels &&
        p.hub_rows >= hub_rows && p.plan_cap >= plan_cap)
        return;
    BC_HIP_TRY(hipStreamSynchronize(st));
    msb_pool_free(p);
    p.n = n;
    p.teams = teams;
    p.wgs = wgs;
    p.cap = cap;
    p.max_levels = max_levels;
    p.hub_rows = hub_rows;
    p.plan_cap = std::max<uint32_t>(plan_cap, 1);
    p.mask_stride = 2 * (uint64_t)n + kStaggerWords / 4;   // even: records stay 16-byte aligned
    p.sig_stride = (uint64_t)n * 64 + 2 * kStaggerWords;
    p.psi_stride = (uint64_t)n * 64 + kStaggerWords;
    p.bnx_stride = (uint64_t)n + kStaggerWords / 8;
    p.cur_stride = (uint64_t)n + kStaggerWords / 16;
    BC_HIP_TRY(hipMalloc((void**)&p.ctl, (size_t)teams * sizeof(TeamCtl)));
    BC_HIP_TRY(hipMalloc((void**)&p.masks, (size_t)teams * p.mask_stride * 8));
    BC_HIP_TRY(hipMalloc((void**)&p.bnx, (size_t)teams * p.bnx_stride * 8));
    BC_HIP_TRY(hipMalloc((void**)&p.cur, (size_t)teams * p.cur_stride * 16));
    BC_HIP_TRY(hipMalloc((void**)&p.sig, (size_t)teams * p.sig_stride * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.psi, (size_t)teams * p.psi_stride * 8));
    BC_HIP_TRY(hipMalloc((void**)&p.hacc, (size_t)wgs * hub_rows * 512));
    BC_HIP_TRY(hipMalloc((void**)&p.lst_v, (size_t)teams * cap * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.bcp, (size_t)teams * cap * 8));
    BC_HIP_TRY(hipMalloc((void**)&p.lst_m, (size_t)teams * cap * 8));
    BC_HIP_TRY(hipMalloc((void**)&p.lvl, (size_t)teams * (max_levels + 2) * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.plan, (size_t)p.plan_cap * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.retry, (size_t)p.plan_cap * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.small, 128 * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.bhist, (size_t)(kPlanBuckets + 1) * 4));
    p.bytes = (size_t)teams * (sizeof(TeamCtl) + 8 * (p.mask_stride + p.bnx_stride + p.psi_stride) +
                               16 * p.cur_stride + 4 * p.sig_stride + 20 * (size_t)cap + 4 * ((size_t)max_levels + 2)) +
              (size_t)wgs * hub_rows * 512 + (size_t)p.plan_cap * 8 + 128 * 4 + (size_t)(kPlanBuckets + 1) * 4;
    if (device >= 0 && device < 64) {
        p.device = device;
        g_pool_bytes[device] += p.bytes;
    }
    const size_t words = (size_t)teams * p.mask_stride;
    const unsigned g1 = (unsigned)std::min<size_t>((words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u64, dim3(g1), dim3(256), 0, st, p.masks, words);
    const size_t bwords = (size_t)teams * p.bnx_stride;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<size_t>((bwords + 255) / 256, 65536)), dim3(256), 0, st,
                       p.bnx, bwords);
    const size_t cwords = (size_t)teams * p.cur_stride * 2;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<size_t>((cwords + 255) / 256, 65536)), dim3(256), 0, st,
                       (uint64_t*)p.cur, cwords);
    const size_t swords = (size_t)teams * p.sig_stride / 2;   // counts, as 64-bit words
    const unsigned g2 = (unsigned)std::min<size_t>((swords + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u64, dim3(g2), dim3(256), 0, st, (uint64_t*)p.sig, swords);
    const size_t cw = (size_t)teams * sizeof(TeamCtl) / 8;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::max<size_t>(1, std::min<size_t>((cw + 255) / 256, 1024))),
                       dim3(256), 0, st, (uint64_t*)p.ctl, cw);
    BC_HIP_TRY(hipGetLastError());
}

// Enqueues the batched path: source plan, batched sweeps, then the per-source kernel on the
// sources handed back.  `retry_launch` enqueues that per-source launch over (list, count).
void run_msb_enqueue(MsbPool& p, const Graph& g, const uint32_t* sources, uint32_t k, double* bc, CallStats* stats,
                     int wg, int team_knob, int slots_cap, int pull16, hipStream_t st, RetryLaunch retry_launch,
                     void* retry_ctx) {
    const DevInfo& di = dev_info(g.device);
    wg = msb_norm_wg(wg);
    const uint32_t n = (uint32_t)g.n;
    const uint32_t active_max = sources ? k : (uint32_t)(g.n - g.zero_out_degree);
    const uint32_t batches = std::max<uint32_t>((active_max + 63) / 64, 1);
    int per_cu = msb_occupancy(wg);
    BC_REQUIRE(per_cu >= 1, BC_E_HIP, "batched kernel does not fit on a compute unit");
    const long max_wgs = (long)per_cu * di.cus;
    // state slots: one per team; the kernel forms min(batches, slots) teams on the device.
    // Unless the caller fixes the team size, a team has at least 4,096 threads, and there are
    // at most a quarter as many slots as compute units: fewer batches in flight keep more of
    // their state in the caches (R-MAT scale 16, 1,024-thread workgroups: 488 GTEPS with one
    // per team, 582 with two, 591 with four; 512-thread workgroups: 96.1, 93.4, 91.4, 94.3 ms
    // with 16, 12, 8, 4 per team), and a slot of a scale-18 graph holds 250 MB, kept by the
    // handle between calls.
    const long slots_max = team_knob > 0 ? max_wgs / team_knob
                                         : std::min<long>(max_wgs / std::max(4, 4096 / wg), di.cus / 4);
    long teams = std::min<long>(batches, std::max<long>(1, slots_max));
    if (slots_cap > 0) teams = std::min<long>(teams, slots_cap);
    const uint32_t cap = (uint32_t)std::min<uint64_t>((uint64_t)n * 8 + 64, 0xffffffffull);
    const uint32_t max_levels = 1024;
    // bound the pool by free device memory (keep half of it for everything else), and the
    // pools of all handles on the device together by three quarters of its memory
    size_t free_b = 0, total_b = 0;
    BC_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const size_t per_team = msb_team_bytes(n, cap, max_levels);
    const size_t have = p.n >= n ? (size_t)p.teams * msb_team_bytes(p.n, p.cap, p.max_levels) : 0;
    const size_t mine = p.device == g.device ? p.bytes : 0;
    const size_t held = g.device >= 0 && g.device < 64 ? g_pool_bytes[g.device].load() : 0;
    const size_t others = held > mine ? held - mine : 0;
    const size_t all = total_b / 4 * 3;
    const size_t room = std::min((free_b + have) / 2, all > others ? all - others : 0);
    const size_t budget = room - std::min<size_t>(room, (size_t)max_wgs * wg * 512);
    teams = (long)std::max<size_t>(1, std::min<size_t>(teams, budget / std::max<size_t>(per_team, 1)));
    const int grid = (int)max_wgs;
    msb_pool_ensure(p, g.device, n, (int)teams, grid, cap, max_levels, (uint32_t)wg, std::max<uint32_t>(k, n), st);

    uint32_t* plan_count = p.small + 80;
    uint32_t* retry_count = p.small + 81;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(128), 0, st, p.small, 128u);
    // the batched kernel runs on the caller's numbering: sources batched by the batching order
    // share more of their rows there than on the copy relabelled by in-degree
    const uint32_t* krow = g.row_ptr;
    const uint32_t* kcol = g.col;
    const uint32_t* kperm = nullptr;
    if (!sources && g.order) {
        const uint32_t active = (uint32_t)(g.n - g.zero_out_degree);
        const unsigned gp = std::max(1u, std::min<unsigned>((active + 255) / 256, 2048));
        hipLaunchKernelGGL(k_plan_all, dim3(gp), dim3(256), 0, st, g.order, n, active, kperm, p.plan, plan_count,
                           stats);
    } else {
        const uint32_t nb = std::min<uint32_t>(n, kPlanBuckets);
        const uint32_t items = sources ? k : n;
        const unsigned gp = std::max(1u, std::min<unsigned>((items + 255) / 256, 2048));
        hipLaunchKernelGGL(k_zero_u32, dim3(std::max(1u, std::min<unsigned>((nb + 256) / 256, 1024))), dim3(256), 0, st,
                           p.bhist, nb + 1);
        hipLaunchKernelGGL(k_plan_hist, dim3(gp), dim3(256), 0, st, g.row_ptr, g.rank, sources, items, n, nb, p.bhist,
                           stats);
        hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, st, p.bhist, nb, plan_count, stats);
        hipLaunchKernelGGL(k_plan_scatter, dim3(gp), dim3(256), 0, st, g.row_ptr, g.rank, sources, items, n, nb,
                           kperm, p.bhist, p.plan);
    }
    BC_HIP_TRY(hipGetLastError());

    MsbArgs a{};
    a.row_ptr = krow;
    a.col = kcol;
    a.bc = bc;
    a.iperm = nullptr;
    a.plan = p.plan;
    a.plan_count = plan_count;
    a.retry = p.retry;
    a.retry_count = retry_count;
    a.stats = stats;
    a.ctl = p.ctl;
    a.masks = p.masks;
    a.sig = p.sig;
    a.psi = p.psi;
    a.bcp = p.bcp;
    a.hacc = p.hacc;
    a.lst_v = p.lst_v;
    a.lst_m = p.lst_m;
    a.lvl = p.lvl;
    a.n = g.n;
    a.mask_stride = p.mask_stride;
    a.sig_stride = p.sig_stride;
    a.psi_stride = p.psi_stride;
    a.cap = p.cap;
    a.max_levels = p.max_levels;
    a.hub_rows = p.hub_rows;
    a.team_size = team_knob > 0 ? (uint32_t)team_knob : 0u;
    a.pool_teams = (uint32_t)std::min<long>(p.teams, teams);   // a reused pool may hold more
    a.sig_cap = g.max_in_degree ? (uint32_t)(0xffffffffull / g.max_in_degree) : 0xffffffffu;
    a.bnx = p.bnx;
    a.bnx_stride = p.bnx_stride;
    if (pull16 > 0) {
        a.csc_ptr = g.csc_ptr;
        a.csc_row = g.csc_row;
        a.cur = p.cur;
        a.cur_stride = p.cur_stride;
        a.pull16 = (uint32_t)pull16;
    }
    // barrier wait bound: 10 s plus 200 ns per vertex and edge of the graph, far above what any
    // level takes (a level reads each out-edge of its entries or each in-edge of the unreached
    // vertices at most once per member's share); only a team whose member stopped making
    // progress reaches it, and the call then fails with BC_E_HIP instead of hanging
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g.device) != hipSuccess || khz <= 0)
            khz = 100000;
        const double secs = 10.0 + 2e-7 * ((double)g.n + (double)g.m);
        a.wait_ticks = (uint64_t)(secs * 1e3 * (double)khz);
    }
    void* args[] = {&a};
    // members of a team wait for each other at level boundaries: a cooperative launch
    // guarantees that every workgroup of the grid is resident at once
    hipError_t e = hipLaunchCooperativeKernel(msb_fn(wg), dim3(grid), dim3(wg), args, 0, st);
    if (e == hipErrorCooperativeLaunchTooLarge) {   // the runtime's residency bound is tighter
        (void)hipGetLastError();
        e = hipLaunchCooperativeKernel(msb_fn(wg), dim3(std::max(1, grid / 2)), dim3(wg), args, 0, st);
    }
    BC_HIP_TRY(e);
    retry_launch(retry_ctx, p.retry, retry_count, std::max<uint32_t>(k, n), false, st);
}

}  // namespace bcmi
