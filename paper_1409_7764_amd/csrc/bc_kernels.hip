// Brandes betweenness centrality, per-source kernels for gfx950.
//
// For one source s (section I, Brandes' method):
//   forward : level-synchronous breadth-first sweep from s.  For frontier vertex v at level d
//             and successor w: the first visitor claims w for level d+1 (compare-and-swap on
//             its distance) and appends it to the next frontier; every edge with
//             dist[w] = d+1 adds sigma[v] into sigma[w] (64-bit integer atomics; a carry out
//             of bit 63 flags the source: its finished levels are converted to double
//             precision and the level being counted is recounted in double precision).
//   backward: levels from the deepest to 0.  Each vertex v of level d owns its own update,
//             pulling from its successors w (dist[w] = d+1):
//                 delta[v] = sigma[v] * sum_w psi[w],   psi[w] = (1 + delta[w]) / sigma[w]
//             which is the successor form of Brandes' dependency recurrence.  No atomics on
//             delta, no predecessor lists (the paper's n^2 predecessor array is replaced by
//             the distance test).  BC[v] += delta[v] for v != s (FP64 atomics).
//
// Scheduling inside a workgroup (one workgroup per source).  A frontier is processed in
// chunks of WG vertices held in LDS.  Per chunk the vertices are classified by out-degree:
//   * hubs (degree >= hub threshold) are cut into pieces of kPiece edges, and each piece is
//     expanded by a whole wavefront: 64 consecutive col[] entries per step, coalesced;
//   * the remaining vertices are expanded either thread-per-vertex (when the chunk's
//     largest degree is small, e.g. lattice-like levels) or thread-per-edge over the
//     chunk's flattened edge list (degree prefix sum in LDS, owner found by binary search),
//     which balances skewed degree mixes.
//
// Two homes for the per-source state:
//   * global memory: one slot per concurrently running source (16-byte {dist, count/psi}
//     record per vertex, BFS queue, level offsets); any graph size;
//   * LDS: the whole state of one source in the workgroup's LDS (12 bytes per vertex:
//     16-bit distance, 64-bit count/psi, 16-bit queue entry) for small graphs.
// Both run the same level code through a small state policy.
#include "bc_internal.h"

#include <algorithm>

namespace bcmi {

namespace {

constexpr uint32_t kPiece = 256;     // hub edges per wavefront work piece
constexpr int kTpv = 4;              // thread-per-vertex mode: chunks whose largest degree is at most this
constexpr int kIlp = 4;              // edges per thread and step in the edge-parallel modes
constexpr double kSafeCount = 1.8e19;   // below 2^64 = 1.8447e19
constexpr uint16_t kUnseen16 = 0xffff;

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ double u2d(uint64_t x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint64_t d2u(double x) { return (uint64_t)__double_as_longlong(x); }

template <class T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x = max(x, (T)__shfl_xor(x, d, 64));
    return x;
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

template <int WG>
struct Scratch {
    uint32_t wsum[3][WG / 64];
    uint32_t scan[WG + 1];     // edge offsets of non-hub vertices in the chunk
    uint32_t pscan[WG + 1];    // piece offsets of hub vertices in the chunk
    uint32_t beg[WG];
    uint32_t deg[WG];
    uint64_t sig[WG];
    double acc[WG];
    uint32_t nq[WG];           // global-memory state: the first WG vertices appended this level
    uint32_t nq_base;          // queue position of nq[0] (the next level's first entry)
    uint32_t tail;             // next free queue position
    uint32_t ovf;              // a 64-bit count carried
    unsigned long long msig;   // largest count of the level being expanded
    uint32_t item, desc;
};

// largest j in [0, WG) with a[j] <= p (a non-decreasing, a[0] = 0 <= p)
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

// Chunk classification: offsets of non-hub edges, offsets of hub pieces, largest non-hub
// degree.  Two block barriers.
template <int WG>
__device__ __forceinline__ void classify_chunk(Scratch<WG>& L, uint32_t deg, bool is_hub, uint32_t& small_off,
                                               uint32_t& small_total, uint32_t& piece_off, uint32_t& piece_total,
                                               uint32_t& max_small) {
    const unsigned lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t a = is_hub ? 0u : deg;
    const uint32_t b = is_hub ? (deg + kPiece - 1) / kPiece : 0u;
    const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
    const uint32_t mx = wave_max(a);
    if (lane == 63) {
        L.wsum[0][w] = ia;
        L.wsum[1][w] = ib;
        L.wsum[2][w] = mx;
    }
    __syncthreads();
    uint32_t ba = 0, bb = 0, ta = 0, tb = 0, tm = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
        const uint32_t x = L.wsum[0][i], y = L.wsum[1][i];
        if (i < (int)w) { ba += x; bb += y; }
        ta += x;
        tb += y;
        tm = max(tm, L.wsum[2][i]);
    }
    small_off = ba + ia - a;
    piece_off = bb + ib - b;
    small_total = ta;
    piece_total = tb;
    max_small = tm;
}

// ---- per-source state policies ------------------------------------------------------------
struct GState {
    static constexpr bool kLdsList = true;       // keep a small next level's vertex list in LDS too
    static constexpr bool kDirectClaim = true;   // thread-per-vertex mode claims without a distance read
    VRec* rec;
    uint32_t* queue;
    uint32_t* lvl;

    __device__ __forceinline__ int claim(uint32_t w, int d1, bool& fresh) {
        fresh = false;
        int dw = rec[w].dist;
        if (dw < 0) {
            const int old = atomicCAS(&rec[w].dist, -1, d1);
            if (old < 0) {
                fresh = true;
                dw = d1;
            } else {
                dw = old;
            }
        }
        return dw;
    }
    __device__ __forceinline__ int dist(uint32_t v) const { return rec[v].dist; }
    __device__ __forceinline__ uint64_t val(uint32_t v) const { return rec[v].val; }
    __device__ __forceinline__ void set_val(uint32_t v, uint64_t x) { rec[v].val = x; }
    __device__ __forceinline__ bool add_u64(uint32_t w, uint64_t s) {
        const unsigned long long old = atomicAdd((unsigned long long*)&rec[w].val, (unsigned long long)s);
        return old + s < old;
    }
    __device__ __forceinline__ void add_u64_nr(uint32_t w, uint64_t s) {
        __hip_atomic_fetch_add((unsigned long long*)&rec[w].val, (unsigned long long)s, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void add_f64(uint32_t w, uint64_t s) { unsafeAtomicAdd((double*)&rec[w].val, u2d(s)); }
    // claim of a vertex whose distance read -1: the CAS decides the first discoverer
    __device__ __forceinline__ int claim_unseen(uint32_t w, int d1, bool& fresh) {
        const int old = atomicCAS(&rec[w].dist, -1, d1);
        fresh = old < 0;
        return fresh ? d1 : old;
    }
    __device__ __forceinline__ double psi_if_level(uint32_t w, int d1) const {
        const VRec r = rec[w];
        return r.dist == d1 ? u2d(r.val) : 0.0;
    }
    __device__ __forceinline__ uint32_t q(uint32_t i) const { return queue[i]; }
    __device__ __forceinline__ void q_set(uint32_t i, uint32_t w) { queue[i] = w; }
    __device__ __forceinline__ void seed(uint32_t s, uint64_t one) {
        rec[s].dist = 0;
        rec[s].val = one;
        queue[0] = s;
        lvl[0] = 0;
        lvl[1] = 1;
    }
    __device__ __forceinline__ void set_level_end(int d, uint32_t end) { lvl[d + 1] = end; }
    __device__ __forceinline__ uint32_t level_begin(int d, uint32_t) const { return lvl[d]; }
    __device__ __forceinline__ void reset(uint32_t v) {
        VRec r;
        r.dist = -1;
        r.pad = 0;
        r.val = 0;
        rec[v] = r;
    }
    // level boundary: make this workgroup's global writes visible to its other waves.  A slot
    // belongs to one workgroup, so workgroup scope is enough; agent scope would write back and
    // invalidate the whole L2 of the XCD at every level.
    __device__ __forceinline__ void barrier() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
};

struct LState {
    static constexpr bool kLdsList = false;      // the queue itself is in LDS
    static constexpr bool kDirectClaim = false;  // distance reads are LDS reads
    uint16_t* dist16;   // 0xffff = not reached
    uint64_t* vals;
    uint16_t* queue;

    __device__ __forceinline__ int claim(uint32_t w, int d1, bool& fresh) {
        fresh = false;
        const uint16_t cur = dist16[w];
        if (cur != kUnseen16) return cur;
        uint32_t* word = reinterpret_cast<uint32_t*>(dist16) + (w >> 1);
        const int sh = (w & 1) * 16;
        uint32_t old = *word;
        for (;;) {
            const uint32_t h = (old >> sh) & 0xffffu;
            if (h != kUnseen16) return (int)h;
            const uint32_t nw = (old & ~(0xffffu << sh)) | ((uint32_t)d1 << sh);
            const uint32_t prev = atomicCAS(word, old, nw);
            if (prev == old) {
                fresh = true;
                return d1;
            }
            old = prev;
        }
    }
    __device__ __forceinline__ int dist(uint32_t v) const {
        const uint16_t d = dist16[v];
        return d == kUnseen16 ? -1 : (int)d;
    }
    __device__ __forceinline__ uint64_t val(uint32_t v) const { return vals[v]; }
    __device__ __forceinline__ void set_val(uint32_t v, uint64_t x) { vals[v] = x; }
    __device__ __forceinline__ bool add_u64(uint32_t w, uint64_t s) {
        const unsigned long long old = atomicAdd((unsigned long long*)&vals[w], (unsigned long long)s);
        return old + s < old;
    }
    __device__ __forceinline__ void add_u64_nr(uint32_t w, uint64_t s) {
        __hip_atomic_fetch_add((unsigned long long*)&vals[w], (unsigned long long)s, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ void add_f64(uint32_t w, uint64_t s) { atomicAdd((double*)&vals[w], u2d(s)); }
    __device__ __forceinline__ int claim_unseen(uint32_t w, int d1, bool& fresh) { return claim(w, d1, fresh); }
    __device__ __forceinline__ double psi_if_level(uint32_t w, int d1) const {
        return dist16[w] == (uint16_t)d1 ? u2d(vals[w]) : 0.0;
    }
    __device__ __forceinline__ uint32_t q(uint32_t i) const { return queue[i]; }
    __device__ __forceinline__ void q_set(uint32_t i, uint32_t w) { queue[i] = (uint16_t)w; }
    __device__ __forceinline__ void seed(uint32_t s, uint64_t one) {
        dist16[s] = 0;
        vals[s] = one;
        queue[0] = (uint16_t)s;
    }
    __device__ __forceinline__ void set_level_end(int, uint32_t) {}
    // the queue is in BFS order, so the levels are contiguous: first entry with dist >= d
    __device__ __forceinline__ uint32_t level_begin(int d, uint32_t hi) const {
        uint32_t lo = 0;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((int)dist16[queue[mid]] < d) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    }
    __device__ __forceinline__ void reset(uint32_t v) {
        dist16[v] = kUnseen16;
        vals[v] = 0;
    }
    __device__ __forceinline__ void barrier() const { __syncthreads(); }
};

// ---- forward sweep ----------------------------------------------------------------------------
// count update of one DAG edge: double precision after a carry; 64-bit without waiting for
// the old value when the level's bound rules out a carry (SAFE); else with the carry check
template <bool F64, bool SAFE, int WG, class S>
__device__ __forceinline__ void add_count(S& st, Scratch<WG>& L, uint32_t w, uint64_t s) {
    if (F64) st.add_f64(w, s);
    else if (SAFE) st.add_u64_nr(w, s);
    else if (st.add_u64(w, s)) L.ovf = 1u;
}

// wavefront-aggregated append of newly discovered vertices to the queue
template <int WG, class S>
__device__ __forceinline__ void append_fresh(S& st, Scratch<WG>& L, bool fresh, uint32_t w) {
    const uint64_t mask = __ballot(fresh);
    if (mask) {
        const unsigned lane = lane_id();
        const unsigned leader = __builtin_ctzll(mask);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&L.tail, (uint32_t)__builtin_popcountll(mask));
        base = __shfl(base, leader, 64);
        if (fresh) {
            const uint32_t pos = base + (uint32_t)__builtin_popcountll(mask & lanemask_lt());
            st.q_set(pos, w);
            if (S::kLdsList && pos - L.nq_base < (uint32_t)WG) L.nq[pos - L.nq_base] = w;
        }
    }
}

// kIlp edges per thread: every distance is read before the first claim, and every claim
// issued before the first count update
template <bool F64, bool SAFE, int WG, class S>
__device__ __forceinline__ void forward_edges(S& st, Scratch<WG>& L, const bool* ok, const uint32_t* w,
                                              const uint64_t* s, int d1, uint32_t& dag) {
    int dw[kIlp];
    bool fresh[kIlp];
#pragma unroll
    for (int t = 0; t < kIlp; ++t) dw[t] = st.dist(w[t]);
#pragma unroll
    for (int t = 0; t < kIlp; ++t) {
        fresh[t] = false;
        if (ok[t] && dw[t] < 0) dw[t] = st.claim_unseen(w[t], d1, fresh[t]);
    }
#pragma unroll
    for (int t = 0; t < kIlp; ++t)
        if (ok[t] && dw[t] == d1) {
            ++dag;
            add_count<F64, SAFE>(st, L, w[t], s[t]);
        }
#pragma unroll
    for (int t = 0; t < kIlp; ++t) append_fresh(st, L, fresh[t], w[t]);
}

template <bool F64, bool SAFE, int WG, class S>
__device__ void expand_level(S& st, Scratch<WG>& L, const uint32_t* __restrict__ row_ptr,
                             const uint32_t* __restrict__ col, uint32_t lo, uint32_t hi, int d, uint32_t hub,
                             uint32_t tpv_max, bool lds_list, uint32_t& exam, uint32_t& dag) {
    const unsigned tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    constexpr unsigned NW = WG / 64;
    const int d1 = d + 1;
    // a level of at most WG vertices was also listed in LDS by the level before (lds_list);
    // its entries are read before the chunk's first barrier, and this level's appends (which
    // rewrite the LDS list) come after it
    for (uint32_t c0 = lo; c0 < hi; c0 += WG) {
        const uint32_t i = c0 + tid;
        const bool valid = i < hi;
        uint32_t v = 0, beg = 0, deg = 0;
        uint64_t sv = 0;
        if (valid) {
            v = lds_list ? L.nq[i - lo] : st.q(i);
            beg = row_ptr[v];
            deg = row_ptr[v + 1] - beg;
            sv = st.val(v);
            exam += deg;
        }
        if (S::kLdsList && tid == 0) L.nq_base = hi;
        const bool is_hub = valid && deg >= hub;
        uint32_t so, stot, po, ptot, mx;
        classify_chunk<WG>(L, deg, is_hub, so, stot, po, ptot, mx);
        if (!F64) {   // the level's largest count bounds the next levels' sums
            const uint64_t ms = wave_max<uint64_t>(valid ? sv : 0ull);
            if (lane == 0 && ms) atomicMax(&L.msig, (unsigned long long)ms);
        }
        if (ptot == 0 && mx <= tpv_max) {
            // thread per vertex, at most kTpv successors each: every successor's distance is
            // read, then every claim issued, before the first count update
            const uint32_t my = is_hub ? 0u : deg;
            uint32_t w[kTpv];
            int dw[kTpv];
            bool fresh[kTpv];
#pragma unroll
            for (int t = 0; t < kTpv; ++t) w[t] = (uint32_t)t < my ? col[beg + t] : 0u;
            if (S::kDirectClaim) {
                // the compare-and-swap returns the distance a plain read would: one round trip
#pragma unroll
                for (int t = 0; t < kTpv; ++t) {
                    fresh[t] = false;
                    dw[t] = (uint32_t)t < my ? st.claim_unseen(w[t], d1, fresh[t]) : 0;
                }
            } else {
#pragma unroll
                for (int t = 0; t < kTpv; ++t) dw[t] = (uint32_t)t < my ? st.dist(w[t]) : 0;
#pragma unroll
                for (int t = 0; t < kTpv; ++t) {
                    fresh[t] = false;
                    if ((uint32_t)t < my && dw[t] < 0) dw[t] = st.claim_unseen(w[t], d1, fresh[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < kTpv; ++t)
                if ((uint32_t)t < my && dw[t] == d1) {
                    ++dag;
                    add_count<F64, SAFE>(st, L, w[t], sv);
                }
#pragma unroll
            for (int t = 0; t < kTpv; ++t) append_fresh(st, L, fresh[t], w[t]);
            __syncthreads();
            continue;
        }
        L.scan[tid] = so;
        L.pscan[tid] = po;
        L.beg[tid] = beg;
        L.deg[tid] = deg;
        L.sig[tid] = sv;
        __syncthreads();
        // thread per edge over the non-hub vertices of the chunk, kIlp edges per thread and
        // step (indices clamped, so every load is issued without a branch around it)
        for (uint32_t p0 = 0; p0 < stot; p0 += kIlp * WG) {
            uint32_t w[kIlp];
            uint64_t s[kIlp];
            bool ok[kIlp];
#pragma unroll
            for (int t = 0; t < kIlp; ++t) {
                const uint32_t p = p0 + t * WG + tid;
                ok[t] = p < stot;
                const uint32_t pc = ok[t] ? p : stot - 1;
                const uint32_t j = find_owner<WG>(L.scan, pc);
                w[t] = col[L.beg[j] + (pc - L.scan[j])];
                s[t] = L.sig[j];
            }
            forward_edges<F64, SAFE>(st, L, ok, w, s, d1, dag);
        }
        // wavefront per hub piece: lanes read 64 consecutive successors per step, kIlp steps
        // at a time
        for (uint32_t pc = wave; pc < ptot; pc += NW) {
            const uint32_t j = find_owner<WG>(L.pscan, pc);
            const uint32_t e0 = (pc - L.pscan[j]) * kPiece;
            const uint32_t e1 = min(L.deg[j], e0 + kPiece);
            const uint32_t b = L.beg[j];
            const uint64_t sj = L.sig[j];
            for (uint32_t e = e0; e < e1; e += 64 * kIlp) {
                uint32_t w[kIlp];
                uint64_t s[kIlp];
                bool ok[kIlp];
#pragma unroll
                for (int t = 0; t < kIlp; ++t) {
                    const uint32_t ee = e + t * 64 + lane;
                    ok[t] = ee < e1;
                    w[t] = col[b + (ok[t] ? ee : e1 - 1)];
                    s[t] = sj;
                }
                forward_edges<F64, SAFE>(st, L, ok, w, s, d1, dag);
            }
        }
        __syncthreads();
    }
}

// ---- backward sweep ---------------------------------------------------------------------------
template <bool F64, int WG, class S>
__device__ void accumulate_level(S& st, Scratch<WG>& L, const uint32_t* __restrict__ row_ptr,
                                 const uint32_t* __restrict__ col, uint32_t lo, uint32_t hi, int d, uint32_t hub,
                                 uint32_t tpv_max, uint32_t src, double* __restrict__ bc, double* ex_delta,
                                 const uint32_t* __restrict__ iperm, double* part) {
    const unsigned tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    constexpr unsigned NW = WG / 64;
    const int d1 = d + 1;
    for (uint32_t c0 = lo; c0 < hi; c0 += WG) {
        const uint32_t i = c0 + tid;
        const bool valid = i < hi;
        uint32_t v = 0, beg = 0, deg = 0;
        uint64_t sv = 0;
        if (valid) {
            v = st.q(i);
            beg = row_ptr[v];
            deg = row_ptr[v + 1] - beg;
            sv = st.val(v);
        }
        double own = 0.0;
        if (part) {
            // deterministic mode: thread per vertex over all of its successors, summed in CSR
            // order (kIlp loads in flight, no atomics)
            for (uint32_t e0 = 0; e0 < deg; e0 += kIlp) {
                uint32_t w[kIlp];
#pragma unroll
                for (int t = 0; t < kIlp; ++t) w[t] = col[beg + min(e0 + (uint32_t)t, deg - 1)];
                double c[kIlp];
#pragma unroll
                for (int t = 0; t < kIlp; ++t) c[t] = st.psi_if_level(w[t], d1);
#pragma unroll
                for (int t = 0; t < kIlp; ++t)
                    if (e0 + (uint32_t)t < deg) own += c[t];
            }
        } else {
        const bool is_hub = valid && deg >= hub;
        uint32_t so, stot, po, ptot, mx;
        classify_chunk<WG>(L, deg, is_hub, so, stot, po, ptot, mx);
        if (ptot == 0 && mx <= tpv_max) {
            // thread per vertex, at most kTpv successors: every successor id, then every
            // successor record, is loaded before the first is used (two round trips, not two per
            // successor); the sum keeps successor order
            const uint32_t my = is_hub ? 0u : deg;
            uint32_t w[kTpv];
#pragma unroll
            for (int t = 0; t < kTpv; ++t) w[t] = (uint32_t)t < my ? col[beg + t] : 0u;
            double c[kTpv];
#pragma unroll
            for (int t = 0; t < kTpv; ++t) c[t] = (uint32_t)t < my ? st.psi_if_level(w[t], d1) : 0.0;
#pragma unroll
            for (int t = 0; t < kTpv; ++t) own += c[t];
        } else {
            L.scan[tid] = so;
            L.pscan[tid] = po;
            L.beg[tid] = beg;
            L.deg[tid] = deg;
            L.acc[tid] = 0.0;
            __syncthreads();
            for (uint32_t p0 = 0; p0 < stot; p0 += kIlp * WG) {   // kIlp edges per thread and step
                uint32_t w[kIlp], jj[kIlp];
                bool ok[kIlp];
#pragma unroll
                for (int t = 0; t < kIlp; ++t) {
                    const uint32_t p = p0 + t * WG + tid;
                    ok[t] = p < stot;
                    const uint32_t pc = ok[t] ? p : stot - 1;
                    jj[t] = find_owner<WG>(L.scan, pc);
                    w[t] = col[L.beg[jj[t]] + (pc - L.scan[jj[t]])];
                }
                double c[kIlp];
#pragma unroll
                for (int t = 0; t < kIlp; ++t) c[t] = st.psi_if_level(w[t], d1);
#pragma unroll
                for (int t = 0; t < kIlp; ++t)
                    if (ok[t] && c[t] != 0.0) atomicAdd(&L.acc[jj[t]], c[t]);
            }
            for (uint32_t pc = wave; pc < ptot; pc += NW) {
                const uint32_t j = find_owner<WG>(L.pscan, pc);
                const uint32_t e0 = (pc - L.pscan[j]) * kPiece;
                const uint32_t e1 = min(L.deg[j], e0 + kPiece);
                const uint32_t b = L.beg[j];
                double part = 0.0;
                for (uint32_t e = e0; e < e1; e += 64 * kIlp) {
                    uint32_t w[kIlp];
                    bool ok[kIlp];
#pragma unroll
                    for (int t = 0; t < kIlp; ++t) {
                        const uint32_t ee = e + t * 64 + lane;
                        ok[t] = ee < e1;
                        w[t] = col[b + (ok[t] ? ee : e1 - 1)];
                    }
                    double c[kIlp];
#pragma unroll
                    for (int t = 0; t < kIlp; ++t) c[t] = st.psi_if_level(w[t], d1);
#pragma unroll
                    for (int t = 0; t < kIlp; ++t)
                        if (ok[t]) part += c[t];
                }
                part = wave_sum(part);
                if (lane == 0 && part != 0.0) atomicAdd(&L.acc[j], part);
            }
            __syncthreads();
            own = L.acc[tid];
        }
        }
        if (valid) {
            const double sigma = F64 ? u2d(sv) : (double)sv;
            const double delta = sigma * own;
            st.set_val(v, d2u((1.0 + delta) / sigma));
            const uint32_t out = iperm ? iperm[v] : v;
            if (v != src && delta != 0.0) {
                if (part)
                    part[out] += delta;   // this workgroup's own array, one owner per vertex and source
                else
                    unsafeAtomicAdd(&bc[out], delta);
            }
            if (ex_delta) ex_delta[out] = delta;
        }
        __syncthreads();
    }
}

// ---- one source -------------------------------------------------------------------------------
template <int WG, class S>
__device__ void one_source(S& st, Scratch<WG>& L, const WorkDesc& D, uint32_t s, const LaunchArgs& a) {
    const unsigned tid = threadIdx.x;
    double* part = a.part ? a.part + (size_t)blockIdx.x * (size_t)D.n : nullptr;   // deterministic mode
    bool f64 = false;
    uint32_t count = 0;
    int nlev = 0;
    uint32_t exam = 0, dag = 0;
    if (tid == 0) {
        st.seed(s, 1ull);
        L.tail = 1;
        L.ovf = 0;
        L.msig = 0;
    }
    uint64_t msig_prev = 1;   // level 0 holds the source, count 1
    const double maxin2 = (double)D.max_in * (double)D.max_in;
    st.barrier();
    uint32_t lo = 0, hi = 1;
    int d = 0;
    bool lds_list = false;   // this level's vertices are also listed in L.nq
    for (;;) {
        // no carry can occur this level if (largest count on level d-1) * maxin^2 < 2^64
        const bool safe = d == 0 || (D.max_in && (double)msig_prev * maxin2 < kSafeCount);
        if (f64)
            expand_level<true, false, WG>(st, L, D.row_ptr, D.col, lo, hi, d, a.hub, a.tpv_max, lds_list, exam, dag);
        else if (safe)
            expand_level<false, true, WG>(st, L, D.row_ptr, D.col, lo, hi, d, a.hub, a.tpv_max, lds_list, exam, dag);
        else
            expand_level<false, false, WG>(st, L, D.row_ptr, D.col, lo, hi, d, a.hub, a.tpv_max, lds_list, exam,
                                           dag);
        st.barrier();
        const uint32_t tail = L.tail;
        const bool ov = L.ovf != 0u;
        msig_prev = L.msig;
        __syncthreads();
        if (tid == 0) L.msig = 0;   // ordered before the next level's updates by its first barrier
        if (!f64 && ov) {
            // A 64-bit sum carried while level d+1 was counted.  Levels 0..d are final and exact:
            // they become doubles; level d+1's partial sums are dropped and recounted in double
            // precision from level d (every vertex of level d+1 is already claimed, so the
            // recount appends nothing; its edges are not counted twice).
            for (uint32_t i = tid; i < hi; i += WG) {
                const uint32_t v = st.q(i);
                st.set_val(v, d2u((double)st.val(v)));
            }
            for (uint32_t i = hi + tid; i < tail; i += WG) st.set_val(st.q(i), 0ull);
            if (tid == 0) L.ovf = 0;
            st.barrier();
            f64 = true;
            uint32_t exam2 = 0, dag2 = 0;
            // level d's list in LDS was overwritten by level d+1's: read the queue
            expand_level<true, false, WG>(st, L, D.row_ptr, D.col, lo, hi, d, a.hub, a.tpv_max, false, exam2, dag2);
            st.barrier();
        }
        if (tail == hi) {
            count = tail;
            break;
        }
        if (tid == 0) st.set_level_end(d + 1, tail);
        lds_list = S::kLdsList && tail - hi <= (uint32_t)WG;   // every entry of level d+1 went to L.nq
        lo = hi;
        hi = tail;
        ++d;
    }
    nlev = d + 1;
    if (a.ex_dist || a.ex_sigma || a.ex_sigma_f) {   // inspection: the forward sweep's result
        for (uint32_t i = tid; i < count; i += WG) {
            const uint32_t v = st.q(i);
            const uint64_t x = st.val(v);
            const uint32_t out = D.iperm ? D.iperm[v] : v;
            if (a.ex_dist) a.ex_dist[out] = st.dist(v);
            if (a.ex_sigma) a.ex_sigma[out] = f64 ? 0ull : x;
            if (a.ex_sigma_f) a.ex_sigma_f[out] = f64 ? u2d(x) : (double)x;
        }
    }
    hi = count;
    for (int dd = nlev - 1; dd >= 0; --dd) {
        lo = st.level_begin(dd, hi);
        if (f64)
            accumulate_level<true, WG>(st, L, D.row_ptr, D.col, lo, hi, dd, a.hub, a.tpv_max, s, D.bc, a.ex_delta,
                                       D.iperm, part);
        else
            accumulate_level<false, WG>(st, L, D.row_ptr, D.col, lo, hi, dd, a.hub, a.tpv_max, s, D.bc, a.ex_delta,
                                        D.iperm, part);
        st.barrier();
        hi = lo;
    }
    for (uint32_t i = tid; i < count; i += WG) st.reset(st.q(i));
    // per-source work counters (examined edges, DAG edges), reduced over the workgroup
    {
        const unsigned lane = lane_id(), w = tid / 64;
        const uint32_t e_w = wave_sum_u32(exam), g_w = wave_sum_u32(dag);
        if (lane == 0) {
            L.wsum[0][w] = e_w;
            L.wsum[1][w] = g_w;
        }
    }
    st.barrier();
    if (tid == 0) {
        uint64_t e_all = 0, g_all = 0;
        for (int i = 0; i < WG / 64; ++i) {
            e_all += L.wsum[0][i];
            g_all += L.wsum[1][i];
        }
        atomicAdd((unsigned long long*)&a.stats->reached, (unsigned long long)count);
        atomicAdd((unsigned long long*)&a.stats->examined, (unsigned long long)e_all);
        atomicAdd((unsigned long long*)&a.stats->dag_edges, (unsigned long long)g_all);
        atomicAdd(&a.stats->n_done, 1u);
        if (f64) atomicAdd(&a.stats->n_overflow, 1u);
        atomicMax(&a.stats->levels_max, (uint32_t)nlev);
        if (f64 && D.ovf_flags) D.ovf_flags[D.iperm ? D.iperm[s] : s] = 1;
        if (D.counters) {
            if (f64) atomicAdd(&D.counters[1], 1u);
            atomicMax(&D.counters[2], (uint32_t)nlev);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(&D.counters[0], 1u);
        }
    }
}

__device__ __forceinline__ uint32_t find_desc(const WorkDesc* descs, uint32_t ndesc, uint32_t item) {
    uint32_t lo = 0, len = ndesc;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (descs[lo + half].item_begin <= item) lo += half;
        len -= half;
    }
    return lo;
}

// claims the next work item for the whole workgroup; false when the list is exhausted
template <int WG>
__device__ __forceinline__ bool claim_item(const LaunchArgs& a, Scratch<WG>& L, uint32_t& di, uint32_t& s,
                                           uint32_t n_cap, uint32_t& seq) {
    const uint32_t total = a.items_dev ? *a.items_dev : a.total_items;
    uint32_t* head = a.head ? a.head : &a.stats->work_head;
    for (;;) {
        if (threadIdx.x == 0) {
            // deterministic mode: a static share, in order (thread 0 keeps the sequence)
            const uint32_t item = a.det ? blockIdx.x + (seq++) * gridDim.x : atomicAdd(head, 1u);
            L.item = item;
            L.desc = item < total ? find_desc(a.descs, a.ndesc, item) : 0u;
        }
        __syncthreads();
        const uint32_t item = L.item;
        di = L.desc;
        __syncthreads();
        if (item >= total) return false;
        const WorkDesc& D = a.descs[di];
        const uint32_t local = item - D.item_begin;
        s = D.sources ? D.sources[local] : D.src_base + local;
        if (s < (uint32_t)D.n && (uint32_t)D.n <= n_cap) {
            if (D.sources && D.perm) s = D.perm[s];   // caller id -> kernel id
            return true;
        }
        if (threadIdx.x == 0) {
            atomicAdd(&a.stats->bad_source, 1u);
            if (D.counters) {
                atomicAdd(&D.counters[3], 1u);
                atomicAdd(&D.counters[0], 1u);
            }
        }
    }
}

template <int WG>
__global__ void __launch_bounds__(WG) k_bc_global(LaunchArgs a) {
    __shared__ Scratch<WG> L;
    GState st;
    st.rec = a.rec + (size_t)blockIdx.x * a.slot_n;
    st.queue = a.queue + (size_t)blockIdx.x * a.slot_n;
    st.lvl = a.lvl + (size_t)blockIdx.x * ((size_t)a.slot_n + 1);
    uint32_t di, s, seq = 0;
    while (claim_item<WG>(a, L, di, s, a.slot_n, seq)) one_source<WG>(st, L, a.descs[di], s, a);
}

template <int WG>
__global__ void __launch_bounds__(WG) k_bc_lds(LaunchArgs a) {
    __shared__ Scratch<WG> L;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t cap = a.lds_n;
    const uint32_t cap2 = (cap + 3) & ~3u;
    LState st;
    st.vals = reinterpret_cast<uint64_t*>(smem);
    st.dist16 = reinterpret_cast<uint16_t*>(smem + 8 * (size_t)cap2);
    st.queue = st.dist16 + cap2;
    for (uint32_t i = threadIdx.x; i < cap2; i += WG) {
        st.vals[i] = 0;
        st.dist16[i] = kUnseen16;
    }
    __syncthreads();
    uint32_t di, s, seq = 0;
    while (claim_item<WG>(a, L, di, s, cap, seq)) one_source<WG>(st, L, a.descs[di], s, a);
}

__global__ void k_prepare(const WorkDesc* descs, uint32_t ndesc, CallStats* stats, uint32_t zero_outputs) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < sizeof(CallStats) / 4)
        reinterpret_cast<uint32_t*>(stats)[threadIdx.x] = 0u;
    if (!zero_outputs) return;
    for (uint32_t d = blockIdx.y; d < ndesc; d += gridDim.y) {
        if (blockIdx.x == 0 && threadIdx.x < 4 && descs[d].counters) descs[d].counters[threadIdx.x] = 0u;
        double* bc = descs[d].bc;
        uint8_t* fl = descs[d].ovf_flags;
        const uint32_t n = (uint32_t)descs[d].n;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            bc[i] = 0.0;
            if (fl) fl[i] = 0;
        }
    }
}

__global__ void k_fill_rec(VRec* rec, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        VRec r;
        r.dist = -1;
        r.pad = 0;
        r.val = 0;
        rec[i] = r;
    }
}

__global__ void k_fill_export(int32_t* dist, uint64_t* sigma, double* sigma_f, double* delta, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (dist) dist[i] = -1;
        if (sigma) sigma[i] = 0;
        if (sigma_f) sigma_f[i] = 0.0;
        if (delta) delta[i] = 0.0;
    }
}

}  // namespace

// ======================================================================================
// host side
// ======================================================================================
namespace {

template <int WG>
void launch_global(const LaunchArgs& a, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_bc_global<WG>, dim3(grid), dim3(WG), 0, st, a);
}
template <int WG>
void launch_lds(const LaunchArgs& a, unsigned grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_bc_lds<WG>, dim3(grid), dim3(WG), lds, st, a);
}

const void* global_fn(int wg) {
    switch (wg) {
        case 64: return (const void*)k_bc_global<64>;
        case 128: return (const void*)k_bc_global<128>;
        case 256: return (const void*)k_bc_global<256>;
        case 512: return (const void*)k_bc_global<512>;
        default: return (const void*)k_bc_global<1024>;
    }
}
const void* lds_fn(int wg) {
    switch (wg) {
        case 64: return (const void*)k_bc_lds<64>;
        case 128: return (const void*)k_bc_lds<128>;
        case 256: return (const void*)k_bc_lds<256>;
        case 512: return (const void*)k_bc_lds<512>;
        default: return (const void*)k_bc_lds<1024>;
    }
}

int norm_wg(int wg) {
    if (wg <= 64) return 64;
    if (wg <= 128) return 128;
    if (wg <= 256) return 256;
    if (wg <= 512) return 512;
    return 1024;
}

}  // namespace

size_t scratch_bytes(int wg) {
    switch (wg) {
        case 64: return sizeof(Scratch<64>);
        case 128: return sizeof(Scratch<128>);
        case 256: return sizeof(Scratch<256>);
        case 512: return sizeof(Scratch<512>);
        default: return sizeof(Scratch<1024>);
    }
}

size_t lds_state_bytes(uint32_t cap) {
    const size_t cap2 = (cap + 3) & ~3u;
    return cap2 * 8 + cap2 * 2 + cap2 * 2;
}

int occupancy_blocks(bool lds_path, int wg, size_t dyn_lds) {
    int per_cu = 0;
    const void* fn = lds_path ? lds_fn(wg) : global_fn(wg);
    if (lds_path && dyn_lds > 0)
        BC_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
    BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, dyn_lds));
    return per_cu;
}

void pool_free(SlotPool& p) {
    if (p.rec) (void)hipFree(p.rec);
    if (p.queue) (void)hipFree(p.queue);
    if (p.lvl) (void)hipFree(p.lvl);
    p = SlotPool{};
}

size_t pool_bytes(uint32_t slot_n, int slots) {
    return (size_t)slots * ((size_t)slot_n * (sizeof(VRec) + 4) + 4 * ((size_t)slot_n + 1));
}

void pool_ensure(SlotPool& p, uint32_t slot_n, int slots, hipStream_t st) {
    if (p.rec && p.slot_n >= slot_n && p.slots >= slots) return;
    BC_HIP_TRY(hipStreamSynchronize(st));
    pool_free(p);
    BC_HIP_TRY(hipMalloc((void**)&p.rec, (size_t)slots * slot_n * sizeof(VRec)));
    BC_HIP_TRY(hipMalloc((void**)&p.queue, (size_t)slots * slot_n * 4));
    BC_HIP_TRY(hipMalloc((void**)&p.lvl, (size_t)slots * ((size_t)slot_n + 1) * 4));
    p.slot_n = slot_n;
    p.slots = slots;
    const size_t count = (size_t)slots * slot_n;
    hipLaunchKernelGGL(k_fill_rec, dim3((unsigned)std::min<size_t>((count + 255) / 256, 65536)), dim3(256), 0, st,
                       p.rec, count);
    BC_HIP_TRY(hipGetLastError());
}

void enqueue_plan(const LaunchPlan& p, hipStream_t st, uint32_t max_n) {
    // zero outputs and counters, then the persistent search kernel
    const unsigned gx = std::max(1u, std::min<unsigned>((max_n + 255) / 256, 1024));
    const unsigned gy = std::max(1u, std::min<unsigned>(p.args.ndesc, 4096));
    hipLaunchKernelGGL(k_prepare, dim3(gx, gy), dim3(256), 0, st, p.args.descs, p.args.ndesc, p.args.stats,
                       p.args.zero_outputs);
    BC_HIP_TRY(hipGetLastError());
    if (p.args.ex_dist || p.args.ex_sigma || p.args.ex_sigma_f || p.args.ex_delta) {
        hipLaunchKernelGGL(k_fill_export, dim3(std::max(1u, std::min<unsigned>((max_n + 255) / 256, 1024))), dim3(256),
                           0, st, p.args.ex_dist, p.args.ex_sigma, p.args.ex_sigma_f, p.args.ex_delta, max_n);
        BC_HIP_TRY(hipGetLastError());
    }
    if ((p.args.total_items == 0 && !p.args.items_dev) || p.grid == 0) return;
    if (p.lds_path) {
        switch (p.wg) {
            case 64: launch_lds<64>(p.args, p.grid, p.dyn_lds, st); break;
            case 128: launch_lds<128>(p.args, p.grid, p.dyn_lds, st); break;
            case 256: launch_lds<256>(p.args, p.grid, p.dyn_lds, st); break;
            case 512: launch_lds<512>(p.args, p.grid, p.dyn_lds, st); break;
            default: launch_lds<1024>(p.args, p.grid, p.dyn_lds, st); break;
        }
    } else {
        switch (p.wg) {
            case 64: launch_global<64>(p.args, p.grid, st); break;
            case 128: launch_global<128>(p.args, p.grid, st); break;
            case 256: launch_global<256>(p.args, p.grid, st); break;
            case 512: launch_global<512>(p.args, p.grid, st); break;
            default: launch_global<1024>(p.args, p.grid, st); break;
        }
    }
    BC_HIP_TRY(hipGetLastError());
}

bool lds_fits(const Knobs& k, uint32_t n, int device) {
    const DevInfo& di = dev_info(device);
    return k.lds_max_n > 0 && n <= (uint32_t)k.lds_max_n && n <= 65535 &&
           lds_state_bytes(n) + scratch_bytes(norm_wg(k.wg_size)) <= (size_t)di.lds_per_block;
}

// Decide path and launch shape for `items` work items over graphs of at most max_n vertices.
LaunchPlan make_plan(const Knobs& k, uint32_t max_n, uint32_t items, int device) {
    LaunchPlan p;
    const DevInfo& di = dev_info(device);
    p.wg = norm_wg(k.wg_size);
    p.lds_path = lds_fits(k, max_n, device);
    p.dyn_lds = p.lds_path ? lds_state_bytes(max_n) : 0;
    int per_cu = occupancy_blocks(p.lds_path, p.wg, p.dyn_lds);
    if (per_cu < 1) {
        BC_REQUIRE(!p.lds_path, BC_E_HIP, "kernel does not fit on a compute unit");
        p.lds_path = false;
        p.dyn_lds = 0;
        per_cu = occupancy_blocks(false, p.wg, 0);
        BC_REQUIRE(per_cu >= 1, BC_E_HIP, "kernel does not fit on a compute unit");
    }
    long grid = (long)per_cu * di.cus;
    if (k.teams > 0) grid = std::min<long>(grid, k.teams);
    grid = std::min<long>(grid, std::max<uint32_t>(items, 1));
    p.grid = (unsigned)std::max<long>(grid, 1);
    p.args.hub = k.hub < 0 ? 0xffffffffu : (uint32_t)std::max(k.hub, 1);
    p.args.tpv_max = kTpv;
    p.args.lds_n = p.lds_path ? max_n : 0;
    p.args.zero_outputs = 1;
    return p;
}

// ---------------------------------------------------------------------------------------
// single-graph entry (exact / sampled / inspection)
// ---------------------------------------------------------------------------------------

struct GraphScratch {
    SlotPool pool;
    WorkDesc* desc = nullptr;    // device, one descriptor
    WorkDesc* rdesc = nullptr;   // device, descriptor of the retry list
    MsbPool* msb = nullptr;
    DeepPool* deep = nullptr;
};

static GraphScratch& scratch_of(Graph& g) {
    if (!g.slots) g.slots = new GraphScratch();
    return *reinterpret_cast<GraphScratch*>(g.slots);
}

void graph_scratch_free(Graph& g) {
    if (!g.slots) return;
    GraphScratch* s = reinterpret_cast<GraphScratch*>(g.slots);
    pool_free(s->pool);
    if (s->desc) (void)hipFree(s->desc);
    if (s->rdesc) (void)hipFree(s->rdesc);
    msb_pool_delete(s->msb);
    deep_pool_delete(s->deep);
    delete s;
    g.slots = nullptr;
}



// Per-source launch over a device-resident list whose length is known only on the device
// (sources the batched kernel handed back).
struct RetryCtx {
    Graph* g;
    GraphScratch* gs;
    Knobs k;
    double* bc;
    uint8_t* ovf_flags;
};

// `kernel_ids`: the list holds ids of the relabelled copy (else caller ids)
static void retry_launch(void* ctx, const uint32_t* list, const uint32_t* count, uint32_t cap, bool kernel_ids,
                         hipStream_t st) {
    RetryCtx& c = *reinterpret_cast<RetryCtx*>(ctx);
    Graph& g = *c.g;
    Knobs k = c.k;
    k.lds_max_n = -1;
    k.teams = 64;
    LaunchPlan p = make_plan(k, (uint32_t)g.n, cap, g.device);
    pool_ensure(c.gs->pool, (uint32_t)g.n, (int)p.grid, st);
    p.args.rec = c.gs->pool.rec;
    p.args.queue = c.gs->pool.queue;
    p.args.lvl = c.gs->pool.lvl;
    p.args.slot_n = c.gs->pool.slot_n;
    WorkDesc d{};
    d.row_ptr = g.krow();
    d.col = g.kcol();
    d.bc = c.bc;
    d.ovf_flags = c.ovf_flags;
    d.sources = list;
    d.perm = kernel_ids ? nullptr : g.perm;
    d.iperm = g.iperm;
    d.n = g.n;
    d.max_in = g.max_in_degree;
    d.num_items = cap;
    BC_HIP_TRY(hipMemcpyAsync(c.gs->rdesc, &d, sizeof(d), hipMemcpyHostToDevice, st));
    p.args.descs = c.gs->rdesc;
    p.args.ndesc = 1;
    p.args.total_items = 0;
    p.args.items_dev = count;
    p.args.head = &g.stats->work_head2;
    p.args.stats = g.stats;
    switch (p.wg) {
        case 64: launch_global<64>(p.args, p.grid, st); break;
        case 128: launch_global<128>(p.args, p.grid, st); break;
        case 256: launch_global<256>(p.args, p.grid, st); break;
        case 512: launch_global<512>(p.args, p.grid, st); break;
        default: launch_global<1024>(p.args, p.grid, st); break;
    }
    BC_HIP_TRY(hipGetLastError());
}

int run_batched(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g);
int run_deep(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g);

// Automatic choice: the batched kernel for graphs beyond the LDS path with at least one full
// batch of sources, unless the graph is deep (most of it lies beyond the batching order's
// ranked levels): a batch then runs past the kernel's level cap and goes to the per-source
// kernel anyway.
static bool want_batched(const Knobs& k, const Graph& g, uint32_t items) {
    if (k.batched < 0 || k.batched >= 2) return false;
    const bool lds_ok = k.lds_max_n > 0 && g.n <= k.lds_max_n;
    if (k.batched > 0) return true;
    return !lds_ok && items >= 64 && !g.deep;
}

// One source per workgroup with its levels in LDS tables (deep.hip).  Switched off: its first
// device run ended in an illegal memory access whose cause has not been shown (a host
// emulation of the same source, under address and thread sanitizers, matches the oracle on
// the same inputs).  The value 2 named an earlier kernel of that kind, removed after a device
// fault.  Asking for either is an error; deep graphs run the global-memory kernel.
static bool want_deep(const Knobs& k, const Graph&) {
    BC_REQUIRE(k.batched != 2, BC_E_INVAL, "batched = 2 (an earlier levels-in-LDS kernel) was removed");
    BC_REQUIRE(k.batched != 3, BC_E_INVAL, "the deep-graph path (batched = 3) is switched off");
    return false;
}

// Descriptor of a one-source-per-workgroup launch over one graph.  Deep graphs keep the
// caller's numbering: a lattice-like graph's own ids put a frontier's neighbours in shared cache
// lines, which the in-degree relabelling would scatter.
WorkDesc single_graph_desc(const Graph& g, const RunArgs& ra) {
    const bool own_ids = g.deep;
    WorkDesc d{};
    d.row_ptr = own_ids ? g.row_ptr : g.krow();
    d.col = own_ids ? g.col : g.kcol();
    d.bc = ra.bc;
    d.ovf_flags = ra.ovf_flags;
    d.sources = ra.sources;
    d.perm = own_ids ? nullptr : g.perm;
    d.iperm = own_ids ? nullptr : g.iperm;
    d.counters = nullptr;
    d.n = g.n;
    d.max_in = g.max_in_degree;
    d.item_begin = 0;
    d.num_items = ra.num_items;
    return d;
}

namespace {
__global__ void k_store_desc(WorkDesc* dst, WorkDesc d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}
}  // namespace

// Writes a descriptor into device memory in stream order, from a kernel argument (no host
// staging buffer).
void store_desc(WorkDesc* dst, const WorkDesc& d, hipStream_t st) {
    hipLaunchKernelGGL(k_store_desc, dim3(1), dim3(64), 0, st, dst, d);
    BC_HIP_TRY(hipGetLastError());
}

// Every record of `count` slot entries back to unreached (distance -1, count 0).
void reset_slot_records(VRec* rec, size_t count, hipStream_t st) {
    if (!count) return;
    hipLaunchKernelGGL(k_fill_rec, dim3((unsigned)std::min<size_t>((count + 255) / 256, 65536)), dim3(256), 0, st,
                       rec, count);
    BC_HIP_TRY(hipGetLastError());
}

namespace {
// BC = the workgroups' partial arrays summed in workgroup order (deterministic mode)
__global__ void k_reduce_parts(const double* __restrict__ part, uint32_t groups, uint32_t n, double* bc) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (uint32_t b = 0; b < groups; ++b) sum += part[(size_t)b * n + v];
        bc[v] = sum;
    }
}
}  // namespace

// Deterministic mode: the global-memory kernel with a static share of the sources per
// workgroup, successor sums in CSR order, and per-workgroup partial BC arrays (at most a
// quarter of free device memory) reduced in workgroup order.
static int run_deterministic(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g) {
    GraphScratch& gs = scratch_of(g);
    if (!gs.desc) BC_HIP_TRY(hipMalloc((void**)&gs.desc, sizeof(WorkDesc)));
    if (!g.stats) BC_HIP_TRY(hipMalloc((void**)&g.stats, sizeof(CallStats)));
    const uint32_t n = (uint32_t)g.n;
    const WorkDesc d = single_graph_desc(g, ra);
    BC_HIP_TRY(hipMemcpyAsync(gs.desc, &d, sizeof(d), hipMemcpyHostToDevice, st));
    Knobs kd = k;
    kd.lds_max_n = -1;   // state in global memory
    LaunchPlan p = make_plan(kd, n, ra.num_items, g.device);
    size_t free_b = 0, total_b = 0;
    BC_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const size_t per = (size_t)n * sizeof(double);
    const size_t fit = std::max<size_t>(1, (free_b / 4) / per);
    p.grid = (unsigned)std::min<size_t>(p.grid, fit);
    pool_ensure(gs.pool, n, (int)p.grid, st);
    p.args.rec = gs.pool.rec;
    p.args.queue = gs.pool.queue;
    p.args.lvl = gs.pool.lvl;
    p.args.slot_n = gs.pool.slot_n;
    p.args.descs = gs.desc;
    p.args.ndesc = 1;
    p.args.total_items = ra.num_items;
    p.args.stats = g.stats;
    double* part = nullptr;
    BC_HIP_TRY(hipMallocAsync((void**)&part, (size_t)p.grid * per, st));
    BC_HIP_TRY(hipMemsetAsync(part, 0, (size_t)p.grid * per, st));
    p.args.part = part;
    p.args.det = 1;
    enqueue_plan(p, st, n);   // zeroes BC and the counters, then the search
    hipLaunchKernelGGL(k_reduce_parts, dim3(std::max(1u, std::min<unsigned>((n + 255) / 256, 4096))), dim3(256), 0,
                       st, part, p.grid, n, ra.bc);
    BC_HIP_TRY(hipGetLastError());
    BC_HIP_TRY(hipFreeAsync(part, st));
    return 0;
}

int run_sources(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g) {
    GraphScratch& gs = scratch_of(g);
    const bool exporting = ra.ex_dist || ra.ex_sigma || ra.ex_sigma_f || ra.ex_delta;
    if (!exporting && k.deterministic) return run_deterministic(ra, k, st, g);
    if (!exporting && want_deep(k, g)) return run_deep(ra, k, st, g);
    if (!exporting && want_batched(k, g, ra.num_items)) return run_batched(ra, k, st, g);
    if (!gs.desc) BC_HIP_TRY(hipMalloc((void**)&gs.desc, sizeof(WorkDesc)));
    if (!g.stats) BC_HIP_TRY(hipMalloc((void**)&g.stats, sizeof(CallStats)));
    const WorkDesc d = single_graph_desc(g, ra);
    BC_HIP_TRY(hipMemcpyAsync(gs.desc, &d, sizeof(d), hipMemcpyHostToDevice, st));

    LaunchPlan p = make_plan(k, (uint32_t)g.n, ra.num_items, g.device);
    if (!p.lds_path) {
        pool_ensure(gs.pool, (uint32_t)g.n, (int)p.grid, st);
        p.args.rec = gs.pool.rec;
        p.args.queue = gs.pool.queue;
        p.args.lvl = gs.pool.lvl;
        p.args.slot_n = gs.pool.slot_n;
    }
    p.args.descs = gs.desc;
    p.args.ndesc = 1;
    p.args.total_items = ra.num_items;
    p.args.stats = g.stats;
    p.args.ex_dist = ra.ex_dist;
    p.args.ex_sigma = ra.ex_sigma;
    p.args.ex_sigma_f = ra.ex_sigma_f;
    p.args.ex_delta = ra.ex_delta;
    enqueue_plan(p, st, (uint32_t)g.n);
    return p.lds_path ? 1 : 0;
}

int run_batched(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g) {
    GraphScratch& gs = scratch_of(g);
    if (!gs.desc) BC_HIP_TRY(hipMalloc((void**)&gs.desc, sizeof(WorkDesc)));
    if (!gs.rdesc) BC_HIP_TRY(hipMalloc((void**)&gs.rdesc, sizeof(WorkDesc)));
    if (!g.stats) BC_HIP_TRY(hipMalloc((void**)&g.stats, sizeof(CallStats)));
    if (!gs.msb) gs.msb = msb_pool_new();
    WorkDesc d{};
    d.row_ptr = g.krow();
    d.col = g.kcol();
    d.bc = ra.bc;
    d.ovf_flags = ra.ovf_flags;
    d.perm = g.perm;
    d.iperm = g.iperm;
    d.n = g.n;
    d.max_in = g.max_in_degree;
    d.num_items = ra.num_items;
    BC_HIP_TRY(hipMemcpyAsync(gs.desc, &d, sizeof(d), hipMemcpyHostToDevice, st));
    // zero BC, the flags and the call counters
    LaunchPlan z;
    z.args.descs = gs.desc;
    z.args.ndesc = 1;
    z.args.total_items = 0;
    z.args.stats = g.stats;
    z.args.zero_outputs = 1;
    z.grid = 0;
    enqueue_plan(z, st, (uint32_t)g.n);
    RetryCtx rc{&g, &gs, k, ra.bc, ra.ovf_flags};
    run_msb_enqueue(*gs.msb, g, ra.sources, ra.num_items, ra.bc, g.stats, k.batch_wg, k.team, k.teams, k.batch_pull,
                    st, retry_launch, &rc);
    return 2;
}

int run_deep(const RunArgs& ra, const Knobs& k, hipStream_t st, Graph& g) {
    GraphScratch& gs = scratch_of(g);
    if (!gs.desc) BC_HIP_TRY(hipMalloc((void**)&gs.desc, sizeof(WorkDesc)));
    if (!gs.rdesc) BC_HIP_TRY(hipMalloc((void**)&gs.rdesc, sizeof(WorkDesc)));
    if (!g.stats) BC_HIP_TRY(hipMalloc((void**)&g.stats, sizeof(CallStats)));
    if (!gs.deep) gs.deep = deep_pool_new();
    WorkDesc d{};
    d.row_ptr = g.row_ptr;
    d.col = g.col;
    d.bc = ra.bc;
    d.ovf_flags = ra.ovf_flags;
    d.n = g.n;
    d.max_in = g.max_in_degree;
    d.num_items = ra.num_items;
    BC_HIP_TRY(hipMemcpyAsync(gs.desc, &d, sizeof(d), hipMemcpyHostToDevice, st));
    // zero BC, the flags and the call counters
    LaunchPlan z;
    z.args.descs = gs.desc;
    z.args.ndesc = 1;
    z.args.total_items = 0;
    z.args.stats = g.stats;
    z.args.zero_outputs = 1;
    z.grid = 0;
    enqueue_plan(z, st, (uint32_t)g.n);
    RetryCtx rc{&g, &gs, k, ra.bc, ra.ovf_flags};
    run_deep_enqueue(*gs.deep, g, ra.sources, ra.num_items, ra.bc, ra.ovf_flags, g.stats, k.teams, st, retry_launch,
                     &rc);
    return 7;
}

// Drops the batched path's state after a team gave up on a barrier (the state is dirty).
void graph_discard_batched_state(Graph& g) {
    if (g.slots) msb_pool_discard(reinterpret_cast<GraphScratch*>(g.slots)->msb);
}

void read_stats(Graph& g, hipStream_t st, CallStats* out) {
    BC_HIP_TRY(hipMemcpyAsync(out, g.stats, sizeof(CallStats), hipMemcpyDeviceToHost, st));
    BC_HIP_TRY(hipStreamSynchronize(st));
}


// ---------------------------------------------------------------------------------------
// batch of independent graphs: one work list over every (graph, source) pair.  Each graph's
// launch knobs are resolved on their own (the autotuner's entry for the graph's size class,
// else the defaults, then the caller's overrides); graphs that share a state home (LDS-resident
// or global slots), workgroup size, hub threshold and grid cap share one persistent launch, and
// inside a launch the graphs run largest work first.  The whole sequence (zeroing, searches) is
// captured once into a hipGraph and replayed while the same graphs, outputs and knobs come back.
// ---------------------------------------------------------------------------------------
struct LaunchKey {
    int lds = 0;      // 1: LDS-resident state
    int wg = 256;
    int hub = 0;
    int teams = 0;    // grid cap (sources per launch), 0 = fill the device
    bool operator==(const LaunchKey& o) const { return lds == o.lds && wg == o.wg && hub == o.hub && teams == o.teams; }
    bool operator<(const LaunchKey& o) const {
        if (lds != o.lds) return lds > o.lds;
        if (wg != o.wg) return wg < o.wg;
        if (hub != o.hub) return hub < o.hub;
        return teams < o.teams;
    }
};

struct BatchPlan {
    int device = 0;
    std::vector<const Graph*> graphs;
    std::vector<uint64_t> uids;       // the graphs' identities (addresses can be reused)
    std::vector<double*> outs;
    std::vector<LaunchKey> keys;      // per graph: the launch it runs in
    bool use_graph = true;
    WorkDesc* d_descs = nullptr;      // [ndesc]
    uint32_t* d_counters = nullptr;   // [ndesc][4]
    CallStats* d_stats = nullptr;     // one per launch
    SlotPool pool;
    std::vector<int> order;           // desc index -> graph index
    std::vector<int> path;            // desc index -> 1 LDS-resident, 0 global slots
    std::vector<LaunchPlan> lp;
    std::vector<uint32_t> maxn;
    hipGraph_t hg = nullptr;
    hipGraphExec_t exec = nullptr;

    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (hg) (void)hipGraphDestroy(hg);
        if (d_descs) (void)hipFree(d_descs);
        if (d_counters) (void)hipFree(d_counters);
        if (d_stats) (void)hipFree(d_stats);
        pool_free(pool);
    }
    bool same(const bc_graph* gs, int num, double* const* bcs, const std::vector<LaunchKey>& k, bool ug,
              int dev) const {
        if (dev != device || num != (int)graphs.size() || ug != use_graph) return false;
        for (int i = 0; i < num; ++i) {
            const Graph* g = (const Graph*)gs[i];
            if (g != graphs[i] || g->uid != uids[i] || bcs[i] != outs[i] || !(k[i] == keys[i])) return false;
        }
        return true;
    }
    bool lists(const Graph* g) const {
        for (size_t i = 0; i < graphs.size(); ++i)
            if (graphs[i] == g && uids[i] == g->uid) return true;
        return false;
    }
};

static std::mutex g_batch_mu;
static BatchPlan* g_batch_plan = nullptr;

static void enqueue_batch(BatchPlan& bp, hipStream_t st) {
    for (size_t c = 0; c < bp.lp.size(); ++c) enqueue_plan(bp.lp[c], st, bp.maxn[c]);
}

// Called when a graph handle is freed: a plan that lists it is dropped before its arrays go.
void batch_forget_graph(const Graph* g) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (g_batch_plan && g_batch_plan->lists(g)) {
        delete g_batch_plan;
        g_batch_plan = nullptr;
    }
}

// The launch each graph of a batch runs in, from its own resolved knobs.
static std::vector<LaunchKey> batch_keys(const bc_graph* gs, int num, const bc_tuning* t, int dev, bool* use_graph) {
    std::vector<LaunchKey> keys(num);
    *use_graph = true;
    for (int i = 0; i < num; ++i) {
        Graph& g = *(Graph*)gs[i];
        const Knobs k = resolve_knobs(g, t);
        keys[i].lds = lds_fits(k, (uint32_t)g.n, dev) ? 1 : 0;
        keys[i].wg = norm_wg(k.wg_size);
        keys[i].hub = k.hub;
        keys[i].teams = k.teams;
        if (i == 0) *use_graph = k.use_graph;
    }
    return keys;
}

static BatchPlan* build_batch_plan(const bc_graph* gs, int num, double* const* bcs, const std::vector<LaunchKey>& keys,
                                   bool use_graph, int dev, hipStream_t st) {
    BatchPlan* bp = new BatchPlan();
    try {
        bp->device = dev;
        bp->keys = keys;
        bp->use_graph = use_graph;
        for (int i = 0; i < num; ++i) {
            bp->graphs.push_back((const Graph*)gs[i]);
            bp->uids.push_back(((const Graph*)gs[i])->uid);
            bp->outs.push_back(bcs[i]);
        }
        // launches: graphs grouped by key, each group largest work first
        std::vector<LaunchKey> uniq(keys.begin(), keys.end());
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        std::vector<std::vector<int>> cls(uniq.size());
        for (int i = 0; i < num; ++i)
            cls[std::lower_bound(uniq.begin(), uniq.end(), keys[i]) - uniq.begin()].push_back(i);
        for (auto& v : cls)
            std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
                const double wa = (double)bp->graphs[a]->n * (bp->graphs[a]->m + 1);
                const double wb = (double)bp->graphs[b]->n * (bp->graphs[b]->m + 1);
                return wa > wb;
            });
        std::vector<WorkDesc> h(num);
        BC_HIP_TRY(hipMalloc((void**)&bp->d_descs, sizeof(WorkDesc) * std::max(num, 1)));
        BC_HIP_TRY(hipMalloc((void**)&bp->d_counters, sizeof(uint32_t) * 4 * std::max(num, 1)));
        BC_HIP_TRY(hipMalloc((void**)&bp->d_stats, sizeof(CallStats) * std::max<size_t>(uniq.size(), 1)));
        int pos = 0;
        uint32_t pool_n = 0;
        long pool_slots = 0;
        std::vector<int> firsts;
        for (size_t c = 0; c < uniq.size(); ++c) {
            const int first = pos;
            uint32_t items = 0, maxn = 0;
            for (int gi : cls[c]) {
                const Graph* g = bp->graphs[gi];
                WorkDesc& d = h[pos];
                d = WorkDesc{};
                d.row_ptr = g->krow();
                d.col = g->kcol();
                d.perm = g->perm;
                d.iperm = g->iperm;
                d.bc = bp->outs[gi];
                d.sources = nullptr;
                d.counters = bp->d_counters + 4 * pos;
                d.n = g->n;
                d.max_in = g->max_in_degree;
                d.item_begin = items;
                d.num_items = (uint32_t)g->n;
                items += (uint32_t)g->n;
                maxn = std::max(maxn, (uint32_t)g->n);
                bp->order.push_back(gi);
                ++pos;
            }
            Knobs kc;
            kc.wg_size = uniq[c].wg;
            kc.hub = uniq[c].hub;
            kc.teams = uniq[c].teams;
            kc.lds_max_n = uniq[c].lds ? (int)std::max<uint32_t>(maxn, 1) : -1;
            LaunchPlan lp = make_plan(kc, maxn, items, dev);
            if (!lp.lds_path) {
                pool_n = std::max(pool_n, maxn);
                pool_slots = std::max<long>(pool_slots, lp.grid);
            }
            lp.args.descs = bp->d_descs + first;
            lp.args.ndesc = (uint32_t)(pos - first);
            lp.args.total_items = items;
            lp.args.stats = bp->d_stats + c;
            bp->path.resize(pos, lp.lds_path ? 1 : 0);
            bp->lp.push_back(lp);
            bp->maxn.push_back(maxn);
        }
        // one slot pool serves every global-slot launch (they run one after another)
        if (pool_slots > 0) pool_ensure(bp->pool, pool_n, (int)pool_slots, st);
        for (LaunchPlan& lp : bp->lp)
            if (!lp.lds_path) {
                lp.args.rec = bp->pool.rec;
                lp.args.queue = bp->pool.queue;
                lp.args.lvl = bp->pool.lvl;
                lp.args.slot_n = bp->pool.slot_n;
            }
        BC_HIP_TRY(hipMemcpyAsync(bp->d_descs, h.data(), sizeof(WorkDesc) * num, hipMemcpyHostToDevice, st));
        BC_HIP_TRY(hipStreamSynchronize(st));
        if (use_graph) {
            hipStream_t cs;
            BC_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                try {
                    enqueue_batch(*bp, cs);
                } catch (...) {
                    hipGraph_t tmp;
                    (void)hipStreamEndCapture(cs, &tmp);
                    if (tmp) (void)hipGraphDestroy(tmp);
                    (void)hipStreamDestroy(cs);
                    throw;
                }
                e = hipStreamEndCapture(cs, &bp->hg);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&bp->exec, bp->hg, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cs);
            BC_HIP_TRY(e);
        }
    } catch (...) {
        delete bp;
        throw;
    }
    return bp;
}

void run_batch(const bc_graph* gs, int num, double* const* bcs, const bc_tuning* t, hipStream_t st, bc_info* infos,
               double* kernel_ms) {
    int dev = 0;
    BC_HIP_TRY(hipGetDevice(&dev));
    bool use_graph = true;
    const std::vector<LaunchKey> keys = batch_keys(gs, num, t, dev, &use_graph);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (!g_batch_plan || !g_batch_plan->same(gs, num, bcs, keys, use_graph, dev)) {
        delete g_batch_plan;
        g_batch_plan = nullptr;
        g_batch_plan = build_batch_plan(gs, num, bcs, keys, use_graph, dev, st);
    }
    BatchPlan& bp = *g_batch_plan;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (infos) {
        BC_HIP_TRY(hipEventCreate(&e0));
        BC_HIP_TRY(hipEventCreate(&e1));
        BC_HIP_TRY(hipEventRecord(e0, st));
    }
    if (bp.exec) BC_HIP_TRY(hipGraphLaunch(bp.exec, st));
    else enqueue_batch(bp, st);
    if (infos) {
        BC_HIP_TRY(hipEventRecord(e1, st));
        BC_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        BC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::vector<uint32_t> cnt(4 * (size_t)num);
        BC_HIP_TRY(hipMemcpy(cnt.data(), bp.d_counters, sizeof(uint32_t) * 4 * num, hipMemcpyDeviceToHost));
        for (int p = 0; p < num; ++p) {
            const int gi = bp.order[p];
            bc_info& inf = infos[gi];
            inf = bc_info{};
            inf.n_sources = cnt[4 * p + 0];
            inf.n_sigma_fp64_fallback = cnt[4 * p + 1];
            inf.levels_max = cnt[4 * p + 2];
            inf.path = (uint32_t)bp.path[p];
            inf.kernel_ms = ms;
            BC_REQUIRE(inf.n_sources == (uint32_t)bp.graphs[gi]->n, BC_E_HIP, "not every source completed");
        }
        if (kernel_ms) *kernel_ms = ms;
    }
}

}  // namespace bcmi
