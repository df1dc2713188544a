// Device code of the deep-graph path: one source per workgroup, each BFS level held in LDS.
//
// Deep graphs (lattices, meshes, road-like graphs) run thousands of levels of tens to hundreds
// of vertices per source.  A level then costs a chain of dependent memory round trips, not
// bandwidth: in the global-memory kernel a queue read, a count read, a distance
// compare-and-swap and a count atomic, the atomics executed beyond the L2.  Here a level keeps
// only two dependent global reads (the out-edges of its vertices, then the reached byte and CSR
// row of each successor, both in small arrays that stay in the caches), and everything else
// happens in LDS.
//
// Method (section I, Brandes; successor form of the dependency recurrence as in the other
// kernels):
//   forward : for v on level d and successor w not reached on levels 0..d,
//             sigma[w] += sigma[v] and w joins level d+1;
//   backward: delta[v] = sigma[v] * (sum over successors w on level d+1 of psi[w]),
//             psi[v] = (1 + delta[v]) / sigma[v];  BC[v] += delta[v] for v != s.
//
// Layout:
//   * LDS, forward: two hash tables (level d, level d+1) keyed by vertex id, each slot
//     {count u64, key u32, CSR begin u32, out-degree u32}, and the listing order of level d.
//     A successor is inserted with an LDS compare-and-swap on its key and counted with an LDS
//     64-bit add that returns the old value (an exact carry test; on a carry the source goes on
//     in double precision);
//   * LDS, backward: three tables {psi f64, key u32} for levels d+1 (read), d (written) and
//     d+2 (cleared for d-1), laid over the same bytes;
//   * global, per slot: a reached byte per vertex (set when a level is listed, cleared by the
//     backward sweep), the level lists in BFS order (vertex, CSR begin, out-degree, count) and
//     the first list entry of each level.
// A level wider than the tables hands the source to the global-memory kernel.
//
// This header holds only device code, so that the same source can be built for a host-side
// emulation of the workgroup (test tooling); deep.hip includes it and adds the launch code.
#pragma once

#include <cstddef>
#include <cstdint>

namespace bcmi {
namespace deep {

constexpr int kWG = 512;                    // workgroup size of the launch
constexpr uint32_t kEmpty = 0xffffffffu;    // free hash slot
constexpr uint32_t kIlp = 4;                // out-edges per thread and step, loads before use

struct Args {
    const uint32_t* row_ptr;   // CSR, caller numbering
    const uint32_t* col;
    double* bc;                // n
    uint8_t* ovf_flags;        // nullable: 1 per source recounted in double precision
    const uint32_t* sources;   // nullable: item i is source i
    uint32_t n;
    uint32_t items;
    uint32_t H;                // hash slots per table
    uint32_t F;                // vertices per level at most (F <= H / 2)
    uint32_t* work_head;       // item counter
    uint32_t* handoffs;        // sources handed to the global-memory kernel (count)
    uint32_t* bad_source;      // sources with id >= n
    uint32_t* retry;           // handed sources (capacity `items`)
    uint64_t* reached;         // call counters (sums over sources)
    uint64_t* examined;
    uint64_t* dag_edges;
    uint32_t* n_done;
    uint32_t* n_overflow;
    uint32_t* levels_max;
    // per-slot state, slot = workgroup
    uint8_t* seen;             // [slots][seen_stride]
    size_t seen_stride;
    uint32_t* lv;              // [slots][list_stride]: level lists, vertex
    uint32_t* lb;              //   CSR begin
    uint32_t* ld;              //   out-degree
    uint64_t* ls;              //   count (u64, or double bits once the source is in double precision)
    size_t list_stride;        // >= n
    uint32_t* lvl;             // [slots][lvl_stride]: first list entry of each level
    size_t lvl_stride;         // >= n + 1
};

// Control words at the start of the dynamic LDS.
struct Ctl {
    uint64_t exam;        // out-edges of the source's reached vertices
    uint64_t dag;         // DAG edges
    uint32_t cnt[2];      // vertices inserted into a level table, by level parity
    uint32_t pos[2];      // listing positions, same parity
    uint32_t full;        // a level outgrew its table
    uint32_t ovf;         // a 64-bit count carried
    uint32_t item;        // broadcast of the claimed work item
    uint32_t pad;
};

// LDS tables after the control words.  Forward: sig[2][H] u64, key[2][H], beg[2][H],
// deg[2][H], idx[F].  Backward: psi[3][H] f64, pkey[3][H], over the same bytes.
struct Lds {
    unsigned char* base;   // 16-byte aligned, after Ctl
    uint32_t H;
    __device__ __forceinline__ uint64_t* sig(uint32_t t) const { return reinterpret_cast<uint64_t*>(base) + (size_t)t * H; }
    __device__ __forceinline__ uint32_t* w32() const { return reinterpret_cast<uint32_t*>(base + 16 * (size_t)H); }
    __device__ __forceinline__ uint32_t* key(uint32_t t) const { return w32() + (size_t)t * H; }
    __device__ __forceinline__ uint32_t* beg(uint32_t t) const { return w32() + (size_t)(2 + t) * H; }
    __device__ __forceinline__ uint32_t* deg(uint32_t t) const { return w32() + (size_t)(4 + t) * H; }
    __device__ __forceinline__ uint32_t* idx() const { return w32() + (size_t)6 * H; }
    __device__ __forceinline__ double* psi(uint32_t t) const { return reinterpret_cast<double*>(base) + (size_t)t * H; }
    __device__ __forceinline__ uint32_t* pkey(uint32_t t) const {
        return reinterpret_cast<uint32_t*>(base + 24 * (size_t)H) + (size_t)t * H;
    }
};

// bytes of dynamic LDS for H slots: control words, forward tables and the listing order
__host__ __device__ constexpr size_t lds_bytes(uint32_t H) {
    return ((sizeof(Ctl) + 15) & ~(size_t)15) + 40 * (size_t)H + 4 * (size_t)(H / 2);
}

__device__ __forceinline__ double u2d(uint64_t x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint64_t d2u(double x) { return (uint64_t)__double_as_longlong(x); }

// Workgroup barrier that also orders global memory: a slot belongs to one workgroup, whose
// waves share one L1, so workgroup scope suffices.
__device__ __forceinline__ void wg_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint32_t hslot(uint32_t w, uint32_t H) {
    return (uint32_t)(((uint64_t)(w * 2654435761u) * H) >> 32);   // multiplicative hash onto [0, H)
}

// slot of w in a table nobody inserts into meanwhile, or H when absent
__device__ __forceinline__ uint32_t hfind(const uint32_t* key, uint32_t H, uint32_t w) {
    uint32_t h = hslot(w, H);
    for (uint32_t i = 0; i < H; ++i) {
        const uint32_t k = key[h];
        if (k == w) return h;
        if (k == kEmpty) return H;
        h = h + 1 == H ? 0u : h + 1;
    }
    return H;
}

// slot of w after inserting it if absent (fresh: this thread inserted it), or H when the
// table is full
__device__ __forceinline__ uint32_t hinsert(uint32_t* key, uint32_t H, uint32_t w, bool& fresh) {
    uint32_t h = hslot(w, H);
    fresh = false;
    for (uint32_t i = 0; i < H; ++i) {
        uint32_t k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmpty) {
            k = atomicCAS(&key[h], kEmpty, w);
            if (k == kEmpty) {
                fresh = true;
                return h;
            }
        }
        if (k == w) return h;
        h = h + 1 == H ? 0u : h + 1;
    }
    return H;
}

// both forward tables empty: keys free, counts zero
template <int WG>
__device__ __forceinline__ void clear_tables(const Lds& T) {
    for (uint32_t i = threadIdx.x; i < 2 * T.H; i += WG) {
        T.key(0)[i] = kEmpty;   // key(1) follows key(0)
        T.sig(0)[i] = 0;        // sig(1) follows sig(0)
    }
}

// raises a control flag (many threads may raise it in one phase; read after the next barrier)
__device__ __forceinline__ void flag(uint32_t& f) {
    __hip_atomic_store(&f, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One out-edge v -> w of a level-d vertex v with count sv.  sn: w's reached byte; rb, re:
// w's CSR row bounds, loaded with it.  Level d+1 goes into table nx.
template <bool F64>
__device__ __forceinline__ void visit(const Lds& T, Ctl& C, const Args& a, uint32_t cur, uint32_t nx, uint32_t w,
                                      uint8_t sn, uint32_t rb, uint32_t re, uint64_t sv, uint32_t& dag) {
    if (sn) return;                                   // reached on a level before d
    if (hfind(T.key(cur), a.H, w) != a.H) return;     // on level d itself
    ++dag;                                            // w is on level d+1: a DAG edge
    bool fresh;
    const uint32_t h = hinsert(T.key(nx), a.H, w, fresh);
    if (h == a.H) {
        flag(C.full);
        return;
    }
    if (fresh) {
        T.beg(nx)[h] = rb;
        T.deg(nx)[h] = re - rb;
        if (atomicAdd(&C.cnt[nx], 1u) >= a.F) flag(C.full);
    }
    if (F64) {
        atomicAdd(reinterpret_cast<double*>(&T.sig(nx)[h]), u2d(sv));
    } else {
        const unsigned long long old =
            atomicAdd(reinterpret_cast<unsigned long long*>(&T.sig(nx)[h]), (unsigned long long)sv);
        if (old + sv < old) flag(C.ovf);
    }
}

// Expansion of level d (table cur, its fc vertices listed in idx) into table nx: thread per
// vertex, kIlp out-edges per step with every successor id, then every reached byte and row
// bound, in flight together.
template <int WG, bool F64>
__device__ __forceinline__ void expand(const Lds& T, Ctl& C, const Args& a, const uint8_t* seen, uint32_t cur,
                                       uint32_t nx, uint32_t fc, uint32_t& exam, uint32_t& dag) {
    const uint32_t* __restrict__ col = a.col;
    const uint32_t* __restrict__ rp = a.row_ptr;
    for (uint32_t i = threadIdx.x; i < fc; i += WG) {
        const uint32_t h = T.idx()[i];
        const uint32_t beg = T.beg(cur)[h], deg = T.deg(cur)[h];
        const uint64_t sv = T.sig(cur)[h];
        exam += deg;
        for (uint32_t t0 = 0; t0 < deg; t0 += kIlp) {
            uint32_t w[kIlp], rb[kIlp], re[kIlp];
            uint8_t sn[kIlp];
#pragma unroll
            for (uint32_t t = 0; t < kIlp; ++t) w[t] = col[beg + min(t0 + t, deg - 1)];
#pragma unroll
            for (uint32_t t = 0; t < kIlp; ++t) {
                sn[t] = seen[w[t]];
                rb[t] = rp[w[t]];
                re[t] = rp[w[t] + 1];
            }
#pragma unroll
            for (uint32_t t = 0; t < kIlp; ++t)
                if (t0 + t < deg) visit<F64>(T, C, a, cur, nx, w[t], sn[t], rb[t], re[t], sv, dag);
        }
    }
}

// Per-slot global state of this workgroup.
struct Slot {
    uint8_t* seen;
    uint32_t* lv;
    uint32_t* lb;
    uint32_t* ld;
    uint64_t* ls;
    uint32_t* lvl;
};

// Backward sweep over the listed levels D..0 (list entries [0, tail)).
template <int WG, bool F64>
__device__ __forceinline__ void backward(const Lds& T, const Args& a, const Slot& S, uint32_t s, int D,
                                         uint32_t tail) {
    const uint32_t H = a.H;
    const uint32_t* __restrict__ col = a.col;
    for (uint32_t i = threadIdx.x; i < 3 * H; i += WG) T.pkey(0)[i] = kEmpty;   // pkey(1), pkey(2) follow
    wg_sync();
    uint32_t hi = tail;
    for (int d = D; d >= 0; --d) {
        const uint32_t lo = S.lvl[d];
        const uint32_t rd = (uint32_t)(d + 1) % 3, wr = (uint32_t)d % 3, cl = (uint32_t)(d + 2) % 3;
        for (uint32_t e = lo + threadIdx.x; e < hi; e += WG) {
            const uint32_t v = S.lv[e], beg = S.lb[e], deg = S.ld[e];
            const uint64_t sv = S.ls[e];
            double sum = 0.0;
            for (uint32_t t0 = 0; t0 < deg; t0 += kIlp) {
                uint32_t w[kIlp];
#pragma unroll
                for (uint32_t t = 0; t < kIlp; ++t) w[t] = col[beg + min(t0 + t, deg - 1)];
#pragma unroll
                for (uint32_t t = 0; t < kIlp; ++t) {
                    if (t0 + t < deg) {
                        const uint32_t h = hfind(T.pkey(rd), H, w[t]);   // w on level d+1: a successor
                        if (h != H) sum += T.psi(rd)[h];
                    }
                }
            }
            const double sigma = F64 ? u2d(sv) : (double)sv;
            const double delta = sigma * sum;
            bool fresh;
            const uint32_t h = hinsert(T.pkey(wr), H, v, fresh);   // a level holds at most F <= H/2 vertices
            if (h != H) T.psi(wr)[h] = (1.0 + delta) / sigma;
            if (v != s && delta != 0.0) unsafeAtomicAdd(&a.bc[v], delta);
            S.seen[v] = 0;
        }
        for (uint32_t h = threadIdx.x; h < H; h += WG) T.pkey(cl)[h] = kEmpty;   // becomes level d-1's table
        wg_sync();
        hi = lo;
    }
}

// One source.  Returns after its contributions are in BC, or after it was handed on.
template <int WG>
__device__ __forceinline__ void one_source(const Lds& T, Ctl& C, const Args& a, const Slot& S, uint32_t s) {
    const unsigned tid = threadIdx.x, lane = tid & 63u;
    const uint32_t H = a.H;
    if (tid == 0) {   // level 0 = {s}, count 1
        const uint32_t b = a.row_ptr[s], dg = a.row_ptr[s + 1] - b;
        const uint32_t h = hslot(s, H);
        T.key(0)[h] = s;
        T.sig(0)[h] = 1ull;
        T.beg(0)[h] = b;
        T.deg(0)[h] = dg;
        T.idx()[0] = h;
        S.lv[0] = s;
        S.lb[0] = b;
        S.ld[0] = dg;
        S.ls[0] = 1ull;
        S.lvl[0] = 0;
        S.seen[s] = 1;
        C.exam = 0;
        C.dag = 0;
        C.cnt[0] = C.cnt[1] = 0;
        C.pos[0] = C.pos[1] = 0;
        C.full = 0;
        C.ovf = 0;
    }
    wg_sync();
    bool f64 = false;
    uint32_t fc = 1, tail = 1;
    uint64_t exam_all = 0, dag_all = 0;   // this thread's share, levels accepted so far
    int d = 0;
    for (;;) {
        const uint32_t cur = (uint32_t)d & 1u, nx = cur ^ 1u;
        uint32_t exam = 0, dag = 0;
        if (f64)
            expand<WG, true>(T, C, a, S.seen, cur, nx, fc, exam, dag);
        else
            expand<WG, false>(T, C, a, S.seen, cur, nx, fc, exam, dag);
        wg_sync();
        const uint32_t nc = C.cnt[nx], full = C.full, ovf = C.ovf;
        if (full || (size_t)tail + nc > a.list_stride || (size_t)d + 2 > a.lvl_stride) {
            // hand the source on: undo the listed levels' reached bytes and both tables
            for (uint32_t e = tid; e < tail; e += WG) S.seen[S.lv[e]] = 0;
            clear_tables<WG>(T);
            if (tid == 0) {
                const uint32_t r = atomicAdd(a.handoffs, 1u);
                if (r < a.items) a.retry[r] = s;
            }
            wg_sync();
            return;
        }
        if (ovf && !f64) {
            // a count passed 2^64: the listed levels and level d go on in double precision,
            // and level d is expanded again.  Every thread has read the control words before
            // they are reset
            wg_sync();
            for (uint32_t e = tid; e < tail; e += WG) S.ls[e] = d2u((double)S.ls[e]);
            for (uint32_t h = tid; h < H; h += WG) {
                if (T.key(cur)[h] != kEmpty) T.sig(cur)[h] = d2u((double)T.sig(cur)[h]);
                T.key(nx)[h] = kEmpty;
                T.sig(nx)[h] = 0;
            }
            if (tid == 0) {
                C.cnt[nx] = 0;
                C.ovf = 0;
            }
            f64 = true;
            wg_sync();
            continue;
        }
        exam_all += exam;
        dag_all += dag;
        if (nc == 0) break;
        // list level d+1 in table order, mark it reached, and free level d's table for d+2
        for (uint32_t h0 = 0; h0 < H; h0 += WG) {
            const uint32_t h = h0 + tid;
            const uint32_t k = h < H ? T.key(nx)[h] : kEmpty;
            const bool occ = k != kEmpty;
            const uint64_t mask = __ballot(occ);
            uint32_t q = 0;
            if (mask) {
                const uint32_t leader = (uint32_t)__builtin_ctzll(mask);
                uint32_t q0 = 0;
                if (lane == leader) q0 = atomicAdd(&C.pos[nx], (uint32_t)__builtin_popcountll(mask));
                q0 = __shfl(q0, (int)leader, 64);
                q = q0 + (uint32_t)__builtin_popcountll(mask & ((1ull << lane) - 1ull));
            }
            if (occ) {
                T.idx()[q] = h;
                const uint32_t e = tail + q;
                S.lv[e] = k;
                S.lb[e] = T.beg(nx)[h];
                S.ld[e] = T.deg(nx)[h];
                S.ls[e] = T.sig(nx)[h];
                S.seen[k] = 1;
            }
            if (h < H) {
                T.key(cur)[h] = kEmpty;
                T.sig(cur)[h] = 0;
            }
        }
        if (tid == 0) {
            S.lvl[d + 1] = tail;
            C.cnt[cur] = 0;
            C.pos[cur] = 0;
        }
        tail += nc;
        fc = nc;
        ++d;
        wg_sync();
    }
    if (f64)
        backward<WG, true>(T, a, S, s, d, tail);
    else
        backward<WG, false>(T, a, S, s, d, tail);
    clear_tables<WG>(T);
    atomicAdd((unsigned long long*)&C.exam, (unsigned long long)exam_all);
    atomicAdd((unsigned long long*)&C.dag, (unsigned long long)dag_all);
    wg_sync();
    if (tid == 0) {
        atomicAdd((unsigned long long*)a.reached, (unsigned long long)tail);
        atomicAdd((unsigned long long*)a.examined, (unsigned long long)C.exam);
        atomicAdd((unsigned long long*)a.dag_edges, (unsigned long long)C.dag);
        atomicAdd(a.n_done, 1u);
        if (f64) {
            atomicAdd(a.n_overflow, 1u);
            if (a.ovf_flags) a.ovf_flags[s] = 1;
        }
        atomicMax(a.levels_max, (uint32_t)(d + 1));
    }
}

// Persistent workgroup of WG threads: claims sources until the items run out.
template <int WG>
__device__ __forceinline__ void worker(const Args& a, unsigned char* smem) {
    Ctl& C = *reinterpret_cast<Ctl*>(smem);
    Lds T;
    T.base = smem + ((sizeof(Ctl) + 15) & ~(size_t)15);
    T.H = a.H;
    Slot S;
    S.seen = a.seen + (size_t)blockIdx.x * a.seen_stride;
    S.lv = a.lv + (size_t)blockIdx.x * a.list_stride;
    S.lb = a.lb + (size_t)blockIdx.x * a.list_stride;
    S.ld = a.ld + (size_t)blockIdx.x * a.list_stride;
    S.ls = a.ls + (size_t)blockIdx.x * a.list_stride;
    S.lvl = a.lvl + (size_t)blockIdx.x * a.lvl_stride;
    clear_tables<WG>(T);
    wg_sync();
    for (;;) {
        if (threadIdx.x == 0) C.item = atomicAdd(a.work_head, 1u);
        wg_sync();
        const uint32_t item = C.item;
        wg_sync();
        if (item >= a.items) break;
        const uint32_t s = a.sources ? a.sources[item] : item;
        if (s >= a.n) {
            if (threadIdx.x == 0) atomicAdd(a.bad_source, 1u);
            continue;
        }
        one_source<WG>(T, C, a, S, s);
    }
}

}  // namespace deep
}  // namespace bcmi
