// One source per workgroup with each BFS level held in LDS: the path for deep graphs
// (lattices, meshes, road-like graphs) whose searches run through thousands of narrow
// levels.  There the time per level, not bandwidth, bounds a search: every level of the
// global-memory kernel waits on a queue read, a count read, a compare-and-swap and a count
// atomic in turn, and on gfx950 the device-wide atomics execute beyond the L2.
//
// The method is unchanged (section I, Brandes' method; successor form of the dependency
// recurrence as in the other kernels):
//   forward : for v on level d and successor w not reached before level d+1,
//             sigma[w] += sigma[v] and w joins level d+1;
//   backward: delta[v] = sigma[v] * sum over successors w on level d+1 of psi[w],
//             psi[w] = (1 + delta[w]) / sigma[w];  BC[v] += delta[v] for v != s.
//
// What moves where:
//   * a level lives in an LDS hash table keyed by vertex id: {key, count, CSR begin,
//     out-degree}.  The next level is built by LDS compare-and-swap on the key and LDS
//     64-bit adds of the counts (returning, so a carry out of bit 63 is seen exactly; the
//     source is then recounted in double precision);
//   * "reached before level d" is a byte per vertex in global memory (`seen`), set when a
//     level is listed and cleared by the backward sweep.  Whether the byte stores of level d
//     are visible yet is never relied on: level d's own table answers for level d;
//   * every level is listed in global memory (vertex, CSR begin, degree, count) for the
//     backward sweep, which keeps psi of level d+1 in a second LDS hash table and looks the
//     successors up there: no distance or count gathers at all;
//   * CSR begin and degree of a candidate successor are loaded together with its `seen`
//     byte, so the next level needs no row-offset round trip.
// A level wider than the table's capacity hands the source to the global-memory kernel.
#include "bc_internal.h"

#include <algorithm>

namespace bcmi {

namespace {

constexpr int kNWG = 256;             // workgroup size
constexpr uint32_t kEmptyKey = 0xffffffffu;
constexpr uint32_t kNarrowTpv = 4;    // forward: thread per vertex up to this level max degree
constexpr uint32_t kNarrowTpvB = 32;  // backward: thread per vertex up to this level max degree
constexpr int kNIlp = 4;              // edges per thread and step in the edge-parallel mode

__device__ __forceinline__ unsigned nlane() { return __lane_id(); }
__device__ __forceinline__ uint64_t nlanemask_lt() { return (1ull << nlane()) - 1ull; }
__device__ __forceinline__ double nu2d(uint64_t x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint64_t nd2u(double x) { return (uint64_t)__double_as_longlong(x); }

__device__ __forceinline__ uint32_t nwave_incl_scan(uint32_t x) {
    const unsigned lane = nlane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}
__device__ __forceinline__ uint32_t nwave_sum(uint32_t x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Workgroup barrier for LDS data only: no wait for outstanding global memory operations.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// Workgroup barrier that also orders global memory: a slot belongs to one workgroup, and the
// waves of a workgroup share one L1, so workgroup scope suffices.
__device__ __forceinline__ void mem_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint32_t hslot(uint32_t w, uint32_t H) {
    return (uint32_t)(((uint64_t)(w * 2654435761u) * H) >> 32);   // multiplicative hash onto [0, H)
}
__device__ __forceinline__ uint32_t hnext(uint32_t h, uint32_t H) { return h + 1 == H ? 0u : h + 1; }

// slot of w in a table nobody writes concurrently, or H when absent
__device__ __forceinline__ uint32_t hfind(const uint32_t* key, uint32_t H, uint32_t w) {
    uint32_t h = hslot(w, H);
    for (uint32_t i = 0; i < H; ++i) {
        const uint32_t k = key[h];
        if (k == w) return h;
        if (k == kEmptyKey) return H;
        h = hnext(h, H);
    }
    return H;
}
// slot of w after inserting it if absent (fresh = this thread inserted it), or H when the
// table is full
__device__ __forceinline__ uint32_t hinsert(uint32_t* key, uint32_t H, uint32_t w, bool& fresh) {
    uint32_t h = hslot(w, H);
    fresh = false;
    for (uint32_t i = 0; i < H; ++i) {
        uint32_t k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmptyKey) {
            k = atomicCAS(&key[h], kEmptyKey, w);
            if (k == kEmptyKey) {
                fresh = true;
                return h;
            }
        }
        if (k == w) return h;
        h = hnext(h, H);
    }
    return H;
}

// largest j in [0, kNWG) with a[j] <= p (a non-decreasing, a[0] = 0 <= p)
__device__ __forceinline__ uint32_t nfind_owner(const uint32_t* a, uint32_t p) {
    uint32_t lo = 0, len = kNWG;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (a[lo + half] <= p) lo += half;
        len -= half;
    }
    return lo;
}

struct NarrowArgs {
    const uint32_t* row_ptr;
    const uint32_t* col;
    double* bc;
    const uint32_t* sources;   // nullable: item i is source i
    uint32_t n;
    uint32_t items;
    uint32_t H;                // hash slots per table
    uint32_t F;                // vertices per level at most (F <= H/2)
    CallStats* stats;
    uint32_t* retry;           // sources handed to the global-memory kernel (capacity `items`)
    // per-slot state, slot = workgroup
    uint8_t* seen;             // [slots][seen_stride]
    size_t seen_stride;
    uint32_t* ev;              // level lists, [slots][n]: vertex
    uint32_t* eb;              //   CSR begin
    uint32_t* ed;              //   out-degree
    uint64_t* es;              //   count (uint64, or double bits after a carry)
    uint2* lvl;                // [slots][n + 2]: {first list entry, largest out-degree} per level
};

// one workgroup's slot
struct NSlot {
    uint8_t* seen;
    uint32_t* ev;
    uint32_t* eb;
    uint32_t* ed;
    uint64_t* es;
    uint2* lvl;
};

struct NShared {
    uint32_t wsum[2][kNWG / 64];
    uint32_t scan[kNWG + 1];
    uint32_t beg[kNWG];
    union {
        uint64_t sig[kNWG];
        double acc[kNWG];
    };
    uint32_t cnt[2];    // vertices inserted into the next table, by parity of the next level
    uint32_t pos[2];    // listing positions, same parity
    uint32_t maxd[2];   // largest out-degree in the next table, same parity
    uint32_t full;      // a level did not fit its table
    uint32_t ovf;       // a 64-bit count carried
    uint32_t item;
    uint32_t sdeg;
};

// LDS tables of one workgroup.  Forward: two level tables (current, next), each
// {count u64, key, CSR begin, degree}, plus the listing order of the current level.
// Backward: three psi tables {psi f64, key} (level d+1 read, level d written, level d+2
// cleared), laid over the same bytes.  Table c is found by offset arithmetic, so the
// accesses stay LDS instructions.
struct Tables {
    unsigned char* base;
    uint32_t H;
    __device__ __forceinline__ uint64_t* sig(uint32_t c) const { return reinterpret_cast<uint64_t*>(base) + (size_t)c * H; }
    __device__ __forceinline__ uint32_t* w32() const { return reinterpret_cast<uint32_t*>(base + 16 * (size_t)H); }
    __device__ __forceinline__ uint32_t* key(uint32_t c) const { return w32() + (size_t)c * H; }
    __device__ __forceinline__ uint32_t* beg(uint32_t c) const { return w32() + (size_t)(2 + c) * H; }
    __device__ __forceinline__ uint32_t* deg(uint32_t c) const { return w32() + (size_t)(4 + c) * H; }
    __device__ __forceinline__ uint32_t* idx() const { return w32() + (size_t)6 * H; }
    __device__ __forceinline__ double* psi(uint32_t c) const { return reinterpret_cast<double*>(base) + (size_t)c * H; }
    __device__ __forceinline__ uint32_t* pkey(uint32_t c) const {
        return reinterpret_cast<uint32_t*>(base + 24 * (size_t)H) + (size_t)c * H;
    }
};

// forward tables back to empty: keys free, counts zero
__device__ __forceinline__ void clear_forward(const Tables& T, uint32_t H) {
    for (uint32_t i = threadIdx.x; i < 2 * H; i += kNWG) {
        T.key(0)[i] = kEmptyKey;   // key[1] follows key[0]
        T.sig(0)[i] = 0;           // sig[1] follows sig[0]
    }
}

// One DAG-candidate edge v -> w of the forward sweep.  sn: w's reached byte; rb/re: w's
// CSR row bounds, loaded with it.
template <bool F64>
__device__ __forceinline__ void visit(const Tables& T, NShared& L, const NarrowArgs& a, uint32_t cur, uint32_t p,
                                      uint32_t w, uint8_t sn, uint32_t rb, uint32_t re, uint64_t sv, uint32_t& dag) {
    if (sn) return;                                    // reached on an earlier level
    if (hfind(T.key(cur), a.H, w) != a.H) return;      // on level d itself
    ++dag;                                             // w is on level d+1
    bool fresh;
    const uint32_t h = hinsert(T.key(cur ^ 1), a.H, w, fresh);
    if (h == a.H) {
        L.full = 1u;
        return;
    }
    if (fresh) {
        T.beg(cur ^ 1)[h] = rb;
        T.deg(cur ^ 1)[h] = re - rb;
        atomicMax(&L.maxd[p], re - rb);
        if (atomicAdd(&L.cnt[p], 1u) >= a.F) L.full = 1u;
    }
    if (F64) {
        atomicAdd(reinterpret_cast<double*>(&T.sig(cur ^ 1)[h]), nu2d(sv));
    } else {
        const unsigned long long old =
            atomicAdd(reinterpret_cast<unsigned long long*>(&T.sig(cur ^ 1)[h]), (unsigned long long)sv);
        if (old + sv < old) L.ovf = 1u;
    }
}

// Expansion of level d (table `cur`, fc vertices listed in T.idx) into table cur^1.
template <bool F64>
__device__ __forceinline__ void expand(const Tables& T, NShared& L, const NarrowArgs& a, const NSlot& S, uint32_t cur, uint32_t p, uint32_t fc,
                       uint32_t maxd, uint32_t& exam, uint32_t& dag) {
    const unsigned tid = threadIdx.x;
    const uint32_t* __restrict__ col = a.col;
    const uint32_t* __restrict__ rp = a.row_ptr;
    if (maxd <= kNarrowTpv) {
        // thread per vertex: all successor ids, then all their reached bytes and row bounds,
        // are in flight together
        for (uint32_t i = tid; i < fc; i += kNWG) {
            const uint32_t h = T.idx()[i];
            const uint32_t beg = T.beg(cur)[h], deg = T.deg(cur)[h];
            const uint64_t sv = T.sig(cur)[h];
            exam += deg;
            if (deg == 0) continue;
            uint32_t w[kNarrowTpv], rb[kNarrowTpv], re[kNarrowTpv];
            uint8_t sn[kNarrowTpv];
#pragma unroll
            for (uint32_t t = 0; t < kNarrowTpv; ++t) w[t] = col[beg + min(t, deg - 1)];
#pragma unroll
            for (uint32_t t = 0; t < kNarrowTpv; ++t) {
                sn[t] = S.seen[w[t]];
                rb[t] = rp[w[t]];
                re[t] = rp[w[t] + 1];
            }
#pragma unroll
            for (uint32_t t = 0; t < kNarrowTpv; ++t)
                if (t < deg) visit<F64>(T, L, a, cur, p, w[t], sn[t], rb[t], re[t], sv, dag);
        }
        return;
    }
    // thread per edge over chunks of kNWG vertices: degree prefix sum in LDS, owner by binary
    // search, kNIlp edges per thread and step
    const unsigned lane = nlane(), wave = tid / 64;
    for (uint32_t c0 = 0; c0 < fc; c0 += kNWG) {
        const uint32_t i = c0 + tid;
        uint32_t beg = 0, deg = 0;
        uint64_t sv = 0;
        if (i < fc) {
            const uint32_t h = T.idx()[i];
            beg = T.beg(cur)[h];
            deg = T.deg(cur)[h];
            sv = T.sig(cur)[h];
            exam += deg;
        }
        const uint32_t inc = nwave_incl_scan(deg);
        if (lane == 63) L.wsum[0][wave] = inc;
        lds_barrier();
        uint32_t base = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < kNWG / 64; ++k) {
            const uint32_t x = L.wsum[0][k];
            if (k < (int)wave) base += x;
            tot += x;
        }
        L.scan[tid] = base + inc - deg;
        L.beg[tid] = beg;
        L.sig[tid] = sv;
        lds_barrier();
        for (uint32_t p0 = 0; p0 < tot; p0 += kNIlp * kNWG) {
            uint32_t w[kNIlp], rb[kNIlp], re[kNIlp];
            uint64_t s[kNIlp];
            uint8_t sn[kNIlp];
            bool ok[kNIlp];
#pragma unroll
            for (int t = 0; t < kNIlp; ++t) {
                const uint32_t q = p0 + t * kNWG + tid;
                ok[t] = q < tot;
                const uint32_t qc = ok[t] ? q : tot - 1;
                const uint32_t j = nfind_owner(L.scan, qc);
                w[t] = col[L.beg[j] + (qc - L.scan[j])];
                s[t] = L.sig[j];
            }
#pragma unroll
            for (int t = 0; t < kNIlp; ++t) {
                sn[t] = S.seen[w[t]];
                rb[t] = rp[w[t]];
                re[t] = rp[w[t] + 1];
            }
#pragma unroll
            for (int t = 0; t < kNIlp; ++t)
                if (ok[t]) visit<F64>(T, L, a, cur, p, w[t], sn[t], rb[t], re[t], s[t], dag);
        }
        lds_barrier();   // before the next chunk rewrites the prefix sums
    }
}

// psi of a finished vertex into the level's table, its dependency into BC, its reached byte
// cleared for the next source
template <bool F64>
__device__ __forceinline__ void finish(const Tables& T, const NarrowArgs& a, const NSlot& S, uint32_t wr, uint32_t v,
                                       uint64_t sv, double sum, uint32_t s) {
    const double sigma = F64 ? nu2d(sv) : (double)sv;
    const double delta = sigma * sum;
    bool fresh;
    const uint32_t h = hinsert(T.pkey(wr), a.H, v, fresh);   // a level holds at most F <= H/2 vertices
    if (h != a.H) T.psi(wr)[h] = (1.0 + delta) / sigma;
    if (v != s && delta != 0.0) unsafeAtomicAdd(&a.bc[v], delta);
    S.seen[v] = 0;
}

// Backward sweep over the listed levels D..0 (list entries [0, tail)).
template <bool F64>
__device__ __forceinline__ void accumulate(const Tables& T, NShared& L, const NarrowArgs& a, const NSlot& S, uint32_t s, int D,
                           uint32_t tail) {
    const unsigned tid = threadIdx.x, lane = nlane(), wave = tid / 64;
    const uint32_t H = a.H;
    const uint32_t* __restrict__ col = a.col;
    uint32_t hi = tail;
    for (int d = D; d >= 0; --d) {
        const uint2 lv = S.lvl[d];
        const uint32_t lo = lv.x, md = lv.y, cnt = hi - lo;
        const uint32_t rd = (uint32_t)(d + 1) % 3, wr = (uint32_t)d % 3, cl = (uint32_t)(d + 2) % 3;
        if (md <= kNarrowTpvB) {
            for (uint32_t i = tid; i < cnt; i += kNWG) {
                const uint32_t e = lo + i;
                const uint32_t v = S.ev[e], beg = S.eb[e], deg = S.ed[e];
                const uint64_t sv = S.es[e];
                double sum = 0.0;
                for (uint32_t t0 = 0; t0 < deg; t0 += kNIlp) {
                    uint32_t w[kNIlp];
#pragma unroll
                    for (uint32_t t = 0; t < (uint32_t)kNIlp; ++t) w[t] = col[beg + min(t0 + t, deg - 1)];
#pragma unroll
                    for (uint32_t t = 0; t < (uint32_t)kNIlp; ++t) {
                        if (t0 + t >= deg) break;
                        const uint32_t h = hfind(T.pkey(rd), H, w[t]);
                        if (h != H) sum += T.psi(rd)[h];
                    }
                }
                finish<F64>(T, a, S, wr, v, sv, sum, s);
            }
        } else {
            // thread per edge over chunks of kNWG vertices, partial sums in LDS
            for (uint32_t c0 = 0; c0 < cnt; c0 += kNWG) {
                const uint32_t i = c0 + tid;
                const bool valid = i < cnt;
                uint32_t v = 0, beg = 0, deg = 0;
                uint64_t sv = 0;
                if (valid) {
                    const uint32_t e = lo + i;
                    v = S.ev[e];
                    beg = S.eb[e];
                    deg = S.ed[e];
                    sv = S.es[e];
                }
                const uint32_t inc = nwave_incl_scan(deg);
                if (lane == 63) L.wsum[0][wave] = inc;
                lds_barrier();
                uint32_t base = 0, tot = 0;
#pragma unroll
                for (int k = 0; k < kNWG / 64; ++k) {
                    const uint32_t x = L.wsum[0][k];
                    if (k < (int)wave) base += x;
                    tot += x;
                }
                L.scan[tid] = base + inc - deg;
                L.beg[tid] = beg;
                L.acc[tid] = 0.0;
                lds_barrier();
                for (uint32_t p0 = 0; p0 < tot; p0 += kNIlp * kNWG) {
                    uint32_t w[kNIlp], jj[kNIlp];
                    bool ok[kNIlp];
#pragma unroll
                    for (int t = 0; t < kNIlp; ++t) {
                        const uint32_t q = p0 + t * kNWG + tid;
                        ok[t] = q < tot;
                        const uint32_t qc = ok[t] ? q : tot - 1;
                        jj[t] = nfind_owner(L.scan, qc);
                        w[t] = col[L.beg[jj[t]] + (qc - L.scan[jj[t]])];
                    }
#pragma unroll
                    for (int t = 0; t < kNIlp; ++t) {
                        if (!ok[t]) continue;
                        const uint32_t h = hfind(T.pkey(rd), H, w[t]);
                        if (h != H) atomicAdd(&L.acc[jj[t]], T.psi(rd)[h]);
                    }
                }
                lds_barrier();
                if (valid) finish<F64>(T, a, S, wr, v, sv, L.acc[tid], s);
                lds_barrier();   // before the next chunk rewrites the partial sums
            }
        }
        for (uint32_t h = tid; h < H; h += kNWG) T.pkey(cl)[h] = kEmptyKey;   // becomes level d-1's table
        lds_barrier();
        hi = lo;
    }
}

// One source: forward with 64-bit counts, again in double precision after a carry; a level
// wider than the tables hands the source back.
__device__ __forceinline__ void narrow_source(const Tables& T, NShared& L, const NarrowArgs& a, const NSlot& S, uint32_t s) {
    const unsigned tid = threadIdx.x;
    const uint32_t H = a.H;
    bool f64 = false;
    uint32_t tail = 1, exam = 0, dag = 0;
    int D = 0;
    for (;;) {
        exam = 0;
        dag = 0;
        if (tid == 0) {   // level 0 = {s}, count 1
            const uint32_t b = a.row_ptr[s], deg = a.row_ptr[s + 1] - b;
            const uint32_t h = hslot(s, H);
            const uint64_t one = f64 ? nd2u(1.0) : 1ull;
            T.key(0)[h] = s;
            T.sig(0)[h] = one;
            T.beg(0)[h] = b;
            T.deg(0)[h] = deg;
            T.idx()[0] = h;
            S.ev[0] = s;
            S.eb[0] = b;
            S.ed[0] = deg;
            S.es[0] = one;
            S.seen[s] = 1;
            S.lvl[0] = make_uint2(0u, deg);
            L.cnt[0] = L.cnt[1] = 0;
            L.pos[0] = L.pos[1] = 0;
            L.maxd[0] = L.maxd[1] = 0;
            L.full = 0;
            L.ovf = 0;
            L.sdeg = deg;
        }
        mem_barrier();
        uint32_t fc = 1, maxd = L.sdeg;
        tail = 1;
        int d = 0;
        bool redo = false, handed = false;
        for (;;) {
            const uint32_t cur = (uint32_t)d & 1u, nx = cur ^ 1u;
            if (f64)
                expand<true>(T, L, a, S, cur, nx, fc, maxd, exam, dag);
            else
                expand<false>(T, L, a, S, cur, nx, fc, maxd, exam, dag);
            mem_barrier();
            const uint32_t nc = L.cnt[nx], full = L.full, ovf = L.ovf, mdn = L.maxd[nx];
            if (full || tail + nc > a.n) {   // the second never holds: every vertex is listed once
                handed = true;
                break;
            }
            if (ovf && !f64) {
                redo = true;
                break;
            }
            if (nc == 0) break;
            // list level d+1 and mark it reached; free the level-d table for level d+2
            for (uint32_t h = tid; h < H; h += kNWG) {
                const uint32_t k = T.key(nx)[h];
                const bool occ = k != kEmptyKey;
                const uint64_t mask = __ballot(occ);
                uint32_t q = 0;
                if (mask) {
                    const unsigned leader = __builtin_ctzll(mask);
                    if (nlane() == leader) q = atomicAdd(&L.pos[nx], (uint32_t)__builtin_popcountll(mask));
                    q = __shfl(q, leader, 64) + (uint32_t)__builtin_popcountll(mask & nlanemask_lt());
                }
                if (occ) {
                    T.idx()[q] = h;
                    const uint32_t e = tail + q;
                    S.ev[e] = k;
                    S.eb[e] = T.beg(nx)[h];
                    S.ed[e] = T.deg(nx)[h];
                    S.es[e] = T.sig(nx)[h];
                    S.seen[k] = 1;
                }
                T.key(cur)[h] = kEmptyKey;
                T.sig(cur)[h] = 0;
            }
            if (tid == 0) {
                S.lvl[d + 1] = make_uint2(tail, mdn);
                L.cnt[cur] = 0;
                L.pos[cur] = 0;
                L.maxd[cur] = 0;
            }
            tail += nc;
            fc = nc;
            maxd = mdn;
            ++d;
            lds_barrier();
        }
        D = d;
        if (!redo && !handed) break;
        // undo: the listed levels' reached bytes and both tables
        for (uint32_t e = tid; e < tail; e += kNWG) S.seen[S.ev[e]] = 0;
        clear_forward(T, H);
        if (handed && tid == 0) {
            const uint32_t r = atomicAdd(&a.stats->handoffs, 1u);
            a.retry[r] = s;
        }
        mem_barrier();
        if (handed) return;
        f64 = true;
    }
    if (tid == 0) S.lvl[D + 1] = make_uint2(tail, 0u);
    for (uint32_t i = tid; i < 3 * H; i += kNWG) T.pkey(0)[i] = kEmptyKey;   // pkey[1], pkey[2] follow
    mem_barrier();
    if (f64)
        accumulate<true>(T, L, a, S, s, D, tail);
    else
        accumulate<false>(T, L, a, S, s, D, tail);
    clear_forward(T, H);
    {
        const unsigned lane = nlane(), w = tid / 64;
        const uint32_t e_w = nwave_sum(exam), g_w = nwave_sum(dag);
        if (lane == 0) {
            L.wsum[0][w] = e_w;
            L.wsum[1][w] = g_w;
        }
    }
    mem_barrier();
    if (tid == 0) {
        uint64_t e_all = 0, g_all = 0;
        for (int i = 0; i < kNWG / 64; ++i) {
            e_all += L.wsum[0][i];
            g_all += L.wsum[1][i];
        }
        atomicAdd((unsigned long long*)&a.stats->reached, (unsigned long long)tail);
        atomicAdd((unsigned long long*)&a.stats->examined, (unsigned long long)e_all);
        atomicAdd((unsigned long long*)&a.stats->dag_edges, (unsigned long long)g_all);
        atomicAdd(&a.stats->n_done, 1u);
        if (f64) atomicAdd(&a.stats->n_overflow, 1u);
        atomicMax(&a.stats->levels_max, (uint32_t)(D + 1));
    }
}

__global__ void __launch_bounds__(kNWG) k_bc_narrow(NarrowArgs a) {
    __shared__ NShared L;
    extern __shared__ __align__(16) unsigned char smem[];
    Tables T;
    T.base = smem;
    T.H = a.H;
    NSlot S;
    S.seen = a.seen + (size_t)blockIdx.x * a.seen_stride;
    S.ev = a.ev + (size_t)blockIdx.x * a.n;
    S.eb = a.eb + (size_t)blockIdx.x * a.n;
    S.ed = a.ed + (size_t)blockIdx.x * a.n;
    S.es = a.es + (size_t)blockIdx.x * a.n;
    S.lvl = a.lvl + (size_t)blockIdx.x * ((size_t)a.n + 2);
    clear_forward(T, a.H);
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) L.item = atomicAdd(&a.stats->work_head, 1u);
        __syncthreads();
        const uint32_t item = L.item;
        __syncthreads();
        if (item >= a.items) break;
        const uint32_t s = a.sources ? a.sources[item] : item;
        if (s >= a.n) {
            if (threadIdx.x == 0) atomicAdd(&a.stats->bad_source, 1u);
            continue;
        }
        narrow_source(T, L, a, S, s);
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
struct NarrowPool {
    uint8_t* seen = nullptr;
    uint32_t* ev = nullptr;
    uint32_t* eb = nullptr;
    uint32_t* ed = nullptr;
    uint64_t* es = nullptr;
    uint2* lvl = nullptr;
    uint32_t* retry = nullptr;
    uint32_t n = 0;
    size_t seen_stride = 0;
    int slots = 0;
    uint32_t retry_cap = 0;
};

NarrowPool* narrow_pool_new() { return new NarrowPool(); }

static void narrow_pool_release(NarrowPool& p) {
    for (void* q : {(void*)p.seen, (void*)p.ev, (void*)p.eb, (void*)p.ed, (void*)p.es, (void*)p.lvl})
        if (q) (void)hipFree(q);
    p.seen = nullptr;
    p.ev = p.eb = p.ed = nullptr;
    p.es = nullptr;
    p.lvl = nullptr;
    p.n = 0;
    p.slots = 0;
}

void narrow_pool_delete(NarrowPool* p) {
    if (!p) return;
    narrow_pool_release(*p);
    if (p->retry) (void)hipFree(p->retry);
    delete p;
}

// device bytes of one slot: reached bytes, the level lists, the level table
size_t narrow_slot_bytes(uint32_t n) {
    return (((size_t)n + 255) & ~(size_t)255) + (size_t)n * (4 + 4 + 4 + 8) + ((size_t)n + 2) * 8;
}

// LDS geometry: table slots H (a multiple of the workgroup size) and level capacity F = H/2,
// as large as lets four workgroups share a compute unit
static void narrow_geometry(int device, uint32_t& H, uint32_t& F, size_t& dyn) {
    const DevInfo& di = dev_info(device);
    const size_t per_wg = (size_t)di.lds_per_cu / 4;
    const size_t stat = sizeof(NShared) + 256;
    const size_t room = per_wg > stat ? per_wg - stat : 0;
    uint32_t h = (uint32_t)(room / 42) / kNWG * kNWG;   // 40 B per slot + 4 B per level entry (F = H/2)
    h = std::max<uint32_t>(h, kNWG);
    H = h;
    F = h / 2;
    dyn = 40 * (size_t)H + 4 * (size_t)F;
}

void run_narrow_enqueue(NarrowPool& p, const Graph& g, const uint32_t* sources, uint32_t k, double* bc,
                        CallStats* stats, int slots_cap, hipStream_t st, RetryLaunch retry_launch, void* retry_ctx) {
    if (k == 0) return;
    uint32_t H, F;
    size_t dyn;
    narrow_geometry(g.device, H, F, dyn);
    int per_cu = 0;
    BC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bc_narrow, kNWG, dyn));
    BC_REQUIRE(per_cu >= 1, BC_E_HIP, "narrow-frontier kernel does not fit on a compute unit");
    long grid = (long)per_cu * dev_info(g.device).cus;
    if (slots_cap > 0) grid = std::min<long>(grid, slots_cap);
    grid = std::min<long>(grid, k);
    const uint32_t n = (uint32_t)g.n;
    if (!p.seen || p.n < n || p.slots < grid) {
        BC_HIP_TRY(hipStreamSynchronize(st));
        narrow_pool_release(p);
        size_t free_b = 0, total_b = 0;
        BC_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        const long fit = (long)((free_b / 2) / narrow_slot_bytes(n));
        BC_REQUIRE(fit >= 1, BC_E_NOMEM, "no room for one narrow-frontier slot");
        const int slots = (int)std::min<long>(grid, fit);
        p.seen_stride = ((size_t)n + 255) & ~(size_t)255;
        BC_HIP_TRY(hipMalloc((void**)&p.seen, p.seen_stride * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.ev, (size_t)n * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.eb, (size_t)n * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.ed, (size_t)n * 4 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.es, (size_t)n * 8 * slots));
        BC_HIP_TRY(hipMalloc((void**)&p.lvl, ((size_t)n + 2) * 8 * slots));
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
    NarrowArgs a{};
    a.row_ptr = g.row_ptr;   // caller numbering: keeps the graph's own locality
    a.col = g.col;
    a.bc = bc;
    a.sources = sources;
    a.n = n;
    a.items = k;
    a.H = H;
    a.F = F;
    a.stats = stats;
    a.retry = p.retry;
    a.seen = p.seen;
    a.seen_stride = p.seen_stride;
    a.ev = p.ev;
    a.eb = p.eb;
    a.ed = p.ed;
    a.es = p.es;
    a.lvl = p.lvl;
    hipLaunchKernelGGL(k_bc_narrow, dim3((unsigned)grid), dim3(kNWG), dyn, st, a);
    BC_HIP_TRY(hipGetLastError());
    // sources whose levels outgrew the tables: the global-memory kernel, same stream
    retry_launch(retry_ctx, p.retry, &stats->handoffs, k, false, st);
}

}  // namespace bcmi
