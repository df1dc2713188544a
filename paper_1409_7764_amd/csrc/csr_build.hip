// CSR / CSC construction on the device from an edge list (section II-D: the pair arrays
// A[i] = u, B[i] = v, converted to the adjacency-list form P/Q with n+1 row offsets).
//
// Steps, all on the device:
//   1. pack   : drop self-loops, flag ids >= n, pack the kept pairs as 64-bit keys u<<b | v
//   2. sort   : least-significant-digit radix sort of the keys, 8-bit digits
//   3. unique : flag first occurrences, exclusive scan -> positions; successor ids to col[],
//               out-degree histogram
//   4. scan   : exclusive scan of the out-degrees -> row_ptr (n+1 entries)
//   5. CSC    : keys v<<b | u of the unique edges, sorted again, giving in-neighbour lists
#include "bc_internal.h"

#include <algorithm>
#include <cstdlib>

namespace bcmi {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;
constexpr int kScanTile = kScanBlock * kScanIpt;

constexpr int kRsBlock = 256;
constexpr int kRsIpt = 16;
constexpr int kRsTile = kRsBlock * kRsIpt;
constexpr int kRsWaves = kRsBlock / 64;

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// inclusive scan across the 64 lanes of a wavefront
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const unsigned lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}

// exclusive scan across the block; returns the block total in *total
__device__ uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const unsigned lane = lane_id();
    const unsigned w = threadIdx.x / 64;
    uint32_t incl = wave_incl_scan(x);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (unsigned i = 0; i < blockDim.x / 64; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tile(const uint32_t* in, uint32_t* out, uint64_t N,
                                                          uint32_t* partials) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanIpt;
    uint32_t v[kScanIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanIpt; ++i) {
        v[i] = (base + i < N) ? in[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(sum, &total);
#pragma unroll
    for (int i = 0; i < kScanIpt; ++i) {
        if (base + i < N) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0 && partials) partials[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(uint32_t* out, uint64_t N, const uint32_t* offs) {
    const uint32_t add = offs[blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock)
        if (base + i < N) out[base + i] += add;
}

// exclusive scan of N uint32 values (in and out may alias)
void scan_u32(const uint32_t* in, uint32_t* out, uint64_t N, hipStream_t st) {
    if (N == 0) return;
    const uint64_t G = (N + kScanTile - 1) / kScanTile;
    if (G == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kScanBlock), 0, st, in, out, N, nullptr);
        BC_HIP_TRY(hipGetLastError());
        return;
    }
    uint32_t* part = nullptr;
    BC_HIP_TRY(hipMallocAsync((void**)&part, G * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)G), dim3(kScanBlock), 0, st, in, out, N, part);
    BC_HIP_TRY(hipGetLastError());
    scan_u32(part, part, G, st);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)G), dim3(kScanBlock), 0, st, out, N, part);
    BC_HIP_TRY(hipGetLastError());
    BC_HIP_TRY(hipFreeAsync(part, st));
}

// --- 1. pack ------------------------------------------------------------------------------
__global__ void k_pack(const uint32_t* src, const uint32_t* dst, uint64_t M, uint32_t n, int vbits,
                       uint64_t* keys, uint32_t* counters /* [0] kept, [1] bad id */) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    uint64_t key = 0;
    if (i < M) {
        const uint32_t u = src[i], v = dst[i];
        if (u >= n || v >= n) {
            atomicOr(&counters[1], 1u);
        } else if (u != v) {
            keep = true;
            key = ((uint64_t)u << vbits) | v;
        }
    }
    const uint64_t mask = __ballot(keep);
    if (mask == 0) return;
    const unsigned lane = lane_id();
    const unsigned leader = __builtin_ctzll(mask);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&counters[0], (uint32_t)__builtin_popcountll(mask));
    base = __shfl(base, leader, 64);
    if (keep) keys[base + __builtin_popcountll(mask & ((1ull << lane) - 1))] = key;
}

// --- 2. radix sort --------------------------------------------------------------------------
__global__ void __launch_bounds__(kRsBlock) k_rs_hist(const uint64_t* keys, uint64_t N, int shift, uint32_t* hist,
                                                      uint32_t G) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += kRsBlock) {
        const uint64_t idx = base + i;
        if (idx < N) atomicAdd(&h[(keys[idx] >> shift) & 0xff], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of one tile are placed in input order within each digit.
__global__ void __launch_bounds__(kRsBlock) k_rs_scatter(const uint64_t* in, uint64_t* out, uint64_t N, int shift,
                                                         const uint32_t* offs, uint32_t G) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kRsWaves][256];
    const unsigned lane = lane_id();
    const unsigned w = threadIdx.x / 64;
    run[threadIdx.x] = offs[(uint64_t)threadIdx.x * G + blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsIpt; ++r) {
#pragma unroll
        for (int q = 0; q < kRsWaves; ++q) wcnt[q][threadIdx.x] = 0;
        __syncthreads();
        const uint64_t idx = base + (uint64_t)r * kRsBlock + threadIdx.x;
        const bool valid = idx < N;
        const uint64_t key = valid ? in[idx] : 0;
        const uint32_t digit = (uint32_t)(key >> shift) & 0xff;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((digit >> b) & 1));
            peers &= ((digit >> b) & 1) ? ones : ~ones;
        }
        const uint32_t rank = __builtin_popcountll(peers & ((1ull << lane) - 1));
        if (valid && rank == 0) wcnt[w][digit] = __builtin_popcountll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[digit] + rank;
            for (unsigned q = 0; q < w; ++q) pos += wcnt[q][digit];
            out[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kRsWaves; ++q) add += wcnt[q][threadIdx.x];
        run[threadIdx.x] += add;
    }
}

// sorts keys[0..N) on bits [0, bits); result returned in whichever buffer holds it
uint64_t* radix_sort(uint64_t* keys, uint64_t* tmp, uint64_t N, int bits, hipStream_t st) {
    if (N <= 1) return keys;
    const uint32_t G = (uint32_t)((N + kRsTile - 1) / kRsTile);
    uint32_t* hist = nullptr;
    BC_HIP_TRY(hipMallocAsync((void**)&hist, (size_t)256 * G * sizeof(uint32_t), st));
    uint64_t* a = keys;
    uint64_t* b = tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(G), dim3(kRsBlock), 0, st, a, N, shift, hist, G);
        BC_HIP_TRY(hipGetLastError());
        scan_u32(hist, hist, (uint64_t)256 * G, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(G), dim3(kRsBlock), 0, st, a, b, N, shift, hist, G);
        BC_HIP_TRY(hipGetLastError());
        std::swap(a, b);
    }
    BC_HIP_TRY(hipFreeAsync(hist, st));
    return a;
}

// --- 3. unique ------------------------------------------------------------------------------
__global__ void k_first_flags(const uint64_t* keys, uint64_t N, uint32_t* flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_unique_scatter(const uint64_t* keys, uint64_t N, const uint32_t* flags, const uint32_t* pos,
                                 int vbits, uint64_t* ukeys, uint32_t* col, uint32_t* deg) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && flags[i]) {
        const uint64_t k = keys[i];
        const uint32_t u = (uint32_t)(k >> vbits);
        const uint32_t v = (uint32_t)(k & ((1ull << vbits) - 1));
        ukeys[pos[i]] = ((uint64_t)v << vbits) | u;   // transposed key, for the CSC sort
        col[pos[i]] = v;
        atomicAdd(&deg[u], 1u);
    }
}

// --- 5. CSC ---------------------------------------------------------------------------------
__global__ void k_csc_fill(const uint64_t* tkeys, uint64_t N, int vbits, uint32_t* row, uint32_t* indeg) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const uint64_t k = tkeys[i];
        row[i] = (uint32_t)(k & ((1ull << vbits) - 1));
        atomicAdd(&indeg[(uint32_t)(k >> vbits)], 1u);
    }
}

__global__ void k_max_u32(const uint32_t* x, uint64_t N, uint32_t* out) {
    uint32_t best = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        best = max(best, x[i]);
    for (int d = 32; d > 0; d >>= 1) best = max(best, (uint32_t)__shfl_xor(best, d, 64));
    if (lane_id() == 0) atomicMax(out, best);
}

// --- 6. relabelling by decreasing in-degree ------------------------------------------------
__global__ void k_degree_keys(const uint32_t* csc_ptr, uint32_t n, uint32_t maxin, int vbits, uint64_t* keys) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        keys[v] = ((uint64_t)(maxin - (csc_ptr[v + 1] - csc_ptr[v])) << vbits) | v;
}

__global__ void k_perm_from_sorted(const uint64_t* keys, uint32_t n, int vbits, uint32_t* iperm, uint32_t* perm) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(keys[i] & ((1ull << vbits) - 1));
        iperm[i] = v;
        perm[v] = i;
    }
}

// relabelled edge keys, one wavefront per row (its lanes stride the row: coalesced, and a
// long row does not hold up a single thread)
__global__ void k_relabel_keys(const uint32_t* row_ptr, const uint32_t* col, uint32_t n, const uint32_t* perm,
                               int vbits, uint64_t* keys) {
    const uint32_t lane = lane_id();
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t u = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; u < n; u += waves) {
        const uint64_t hi = (uint64_t)perm[u] << vbits;
        const uint32_t e1 = row_ptr[u + 1];
        for (uint32_t e = row_ptr[u] + lane; e < e1; e += 64) keys[e] = hi | perm[col[e]];
    }
}

__global__ void k_csr_from_sorted(const uint64_t* keys, uint64_t m, int vbits, uint32_t* col) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        col[i] = (uint32_t)(keys[i] & ((1ull << vbits) - 1));
}

// out-degree of relabelled vertex i: the original vertex's, read from its row offsets
__global__ void k_relabel_degrees(const uint32_t* row_ptr, const uint32_t* iperm, uint32_t n, uint32_t* deg) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t v = iperm[i];
        deg[i] = row_ptr[v + 1] - row_ptr[v];
    }
}

// vertices with no out-edges (row_ptr still holds out-degrees)
__global__ void k_count_zero(const uint32_t* deg, uint64_t N, uint32_t* out) {
    uint32_t c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        c += deg[i] == 0 ? 1u : 0u;
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

// --- 7. batching order ---------------------------------------------------------------------
// Sources batched together gain when their shortest-path DAGs share edges.  The order ranks
// vertices outward from a hub h (largest in-degree among vertices with out-edges) over reversed
// edges: level k holds the vertices at distance k from h, ranked after every lower level, by
// (lowest rank among their successors on level k-1, out-degree bucket, id).  Sources whose
// paths towards h run through the same vertices then sit next to each other, and so do sources
// with a common successor.  Vertices that do not reach h within kOrderLevels come last, by
// out-degree bucket (out-degree 0 last of all).
constexpr uint32_t kInf = 0xffffffffu;
constexpr int kOrderLevels = 64;

__device__ __forceinline__ uint32_t deg_bucket(uint32_t deg) { return deg ? (uint32_t)__clz(deg) : 32u; }

__global__ void k_hub_key(const uint32_t* row_ptr, const uint32_t* csc_ptr, uint32_t n, unsigned long long* best) {
    unsigned long long b = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (row_ptr[v + 1] > row_ptr[v]) {
            const unsigned long long key = ((unsigned long long)(csc_ptr[v + 1] - csc_ptr[v]) << 32) | (kInf - v);
            b = key > b ? key : b;
        }
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long y = (unsigned long long)__shfl_xor((long long)b, d, 64);
        b = y > b ? y : b;
    }
    if (lane_id() == 0 && b) atomicMax(best, b);
}

__global__ void k_order_init(uint32_t* hdist, uint32_t* rank, uint32_t* order, uint32_t n,
                             const unsigned long long* best, uint32_t* frontier) {
    const uint32_t hub = kInf - (uint32_t)(*best & 0xffffffffull);
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        hdist[v] = v == hub ? 0u : kInf;
        rank[v] = v == hub ? 0u : kInf;
        if (v == hub) {
            order[0] = hub;
            frontier[0] = hub;
        }
    }
}

// one wavefront per frontier vertex u: claims its unvisited predecessors for level k
__global__ void k_order_discover(const uint32_t* csc_ptr, const uint32_t* csc_row, const uint32_t* frontier,
                                 uint32_t nf, uint32_t k, uint32_t* hdist, uint32_t* next, uint32_t* next_count) {
    const unsigned lane = lane_id();
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t i = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < nf; i += waves) {
        const uint32_t u = frontier[i];
        for (uint32_t e0 = csc_ptr[u]; e0 < csc_ptr[u + 1]; e0 += 64) {
            const uint32_t e = e0 + lane;
            bool take = false;
            uint32_t v = 0;
            if (e < csc_ptr[u + 1]) {
                v = csc_row[e];
                take = hdist[v] == kInf && atomicCAS(&hdist[v], kInf, k) == kInf;
            }
            const uint64_t mask = __ballot(take);
            if (mask) {
                const unsigned leader = __builtin_ctzll(mask);
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(next_count, (uint32_t)__builtin_popcountll(mask));
                base = __shfl(base, leader, 64);
                if (take) next[base + __builtin_popcountll(mask & ((1ull << lane) - 1))] = v;
            }
        }
    }
}

__global__ void k_order_keys(const uint32_t* row_ptr, const uint32_t* col, const uint32_t* level,
                             const uint32_t* count, uint32_t k, const uint32_t* hdist, const uint32_t* rank, int vbits,
                             uint64_t* keys) {
    const uint32_t nl = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
        const uint32_t v = level[i];
        uint32_t best = kInf;
        for (uint32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const uint32_t u = col[e];
            if (hdist[u] == k - 1) best = min(best, rank[u]);
        }
        const uint32_t deg = row_ptr[v + 1] - row_ptr[v];
        keys[i] = ((uint64_t)best << (vbits + 6)) | ((uint64_t)deg_bucket(deg) << vbits) | v;
    }
}

// the vertices left without a rank, keyed by out-degree bucket
__global__ void k_order_rest(const uint32_t* row_ptr, const uint32_t* rank, uint32_t n, int vbits, uint64_t* keys,
                             uint32_t* count) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (rank[v] == kInf) keys[atomicAdd(count, 1u)] = ((uint64_t)deg_bucket(row_ptr[v + 1] - row_ptr[v]) << vbits) | v;
}

__global__ void k_order_assign(const uint64_t* keys, const uint32_t* count, uint32_t base, int vbits, uint32_t* rank,
                               uint32_t* order, uint32_t* frontier) {
    const uint32_t nl = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(keys[i] & ((1ull << vbits) - 1));
        rank[v] = base + i;
        order[base + i] = v;
        if (frontier) frontier[i] = v;
    }
}

inline unsigned grid_for(uint64_t N, int block) { return (unsigned)std::max<uint64_t>(1, (N + block - 1) / block); }

}  // namespace

// Ranks the vertices for batching (see the batching order above): g.rank[v] and g.order,
// the vertices in rank order.  Needs the CSR and CSC; ids of up to 29 bits.
static void build_order(Graph& g, int vbits, hipStream_t st) {
    const uint32_t n = (uint32_t)g.n;
    if (g.m == 0 || 2 * vbits + 6 > 64) return;
    BC_HIP_TRY(hipMalloc((void**)&g.rank, sizeof(uint32_t) * n));
    BC_HIP_TRY(hipMalloc((void**)&g.order, sizeof(uint32_t) * n));
    uint32_t *hdist = nullptr, *fa = nullptr, *fb = nullptr, *cnt = nullptr;
    uint64_t *ka = nullptr, *kb = nullptr;
    BC_HIP_TRY(hipMallocAsync((void**)&hdist, sizeof(uint32_t) * n, st));
    BC_HIP_TRY(hipMallocAsync((void**)&fa, sizeof(uint32_t) * n, st));
    BC_HIP_TRY(hipMallocAsync((void**)&fb, sizeof(uint32_t) * n, st));
    BC_HIP_TRY(hipMallocAsync((void**)&ka, sizeof(uint64_t) * n, st));
    BC_HIP_TRY(hipMallocAsync((void**)&kb, sizeof(uint64_t) * n, st));
    BC_HIP_TRY(hipMallocAsync((void**)&cnt, sizeof(uint32_t) * 4 * (kOrderLevels + 2), st));
    BC_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * 4 * (kOrderLevels + 2), st));
    unsigned long long* best = (unsigned long long*)cnt;   // cnt[0..1]
    const unsigned gn = std::min<unsigned>(grid_for(n, 256), 4096);
    hipLaunchKernelGGL(k_hub_key, dim3(gn), dim3(256), 0, st, g.row_ptr, g.csc_ptr, n, best);
    hipLaunchKernelGGL(k_order_init, dim3(gn), dim3(256), 0, st, hdist, g.rank, g.order, n, best, fa);
    BC_HIP_TRY(hipGetLastError());
    uint32_t placed = 1, nf = 1;
    // level k's size lands in cnt[2 + k]
    for (uint32_t k = 1; k <= (uint32_t)kOrderLevels && nf > 0; ++k) {
        uint32_t* c = cnt + 2 + k;
        const unsigned gd = std::min<unsigned>(std::max<unsigned>(1, (nf + 3) / 4), 8192);
        hipLaunchKernelGGL(k_order_discover, dim3(gd), dim3(256), 0, st, g.csc_ptr, g.csc_row, fa, nf, k, hdist, fb, c);
        BC_HIP_TRY(hipGetLastError());
        uint32_t nl = 0;
        BC_HIP_TRY(hipMemcpyAsync(&nl, c, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipStreamSynchronize(st));
        if (nl == 0) break;
        const unsigned gl = std::min<unsigned>(grid_for(nl, 256), 4096);
        hipLaunchKernelGGL(k_order_keys, dim3(gl), dim3(256), 0, st, g.row_ptr, g.col, fb, c, k, hdist, g.rank, vbits, ka);
        BC_HIP_TRY(hipGetLastError());
        uint64_t* sorted = radix_sort(ka, kb, nl, 2 * vbits + 6, st);
        hipLaunchKernelGGL(k_order_assign, dim3(gl), dim3(256), 0, st, sorted, c, placed, vbits, g.rank, g.order, fa);
        BC_HIP_TRY(hipGetLastError());
        placed += nl;
        nf = nl;
    }
    g.deep = (uint64_t)placed * 2 < (uint64_t)(n - g.zero_out_degree);
    if (placed < n) {
        uint32_t* c = cnt + 2 + kOrderLevels + 1;
        BC_HIP_TRY(hipMemsetAsync(c, 0, sizeof(uint32_t), st));
        hipLaunchKernelGGL(k_order_rest, dim3(gn), dim3(256), 0, st, g.row_ptr, g.rank, n, vbits, ka, c);
        BC_HIP_TRY(hipGetLastError());
        uint64_t* sorted = radix_sort(ka, kb, n - placed, vbits + 6, st);
        hipLaunchKernelGGL(k_order_assign, dim3(gn), dim3(256), 0, st, sorted, c, placed, vbits, g.rank, g.order,
                           (uint32_t*)nullptr);
        BC_HIP_TRY(hipGetLastError());
    }
    for (void* q : {(void*)hdist, (void*)fa, (void*)fb, (void*)ka, (void*)kb, (void*)cnt}) BC_HIP_TRY(hipFreeAsync(q, st));
}

void build_csr_device(int32_t n, int64_t m_in, const uint32_t* d_src, const uint32_t* d_dst, hipStream_t st,
                      Graph& g) {
    BC_REQUIRE(n >= 1, BC_E_RANGE, "n must be >= 1");
    BC_REQUIRE(m_in >= 0, BC_E_INVAL, "m_in must be >= 0");
    BC_REQUIRE(m_in < (int64_t)0xffffffffLL, BC_E_RANGE, "more than 2^32-2 input pairs");
    BC_REQUIRE(m_in == 0 || (d_src && d_dst), BC_E_INVAL, "null edge arrays");
    const uint64_t M = (uint64_t)m_in;
    int vbits = 1;
    while (vbits < 31 && (1ull << vbits) < (uint64_t)n) ++vbits;

    g.n = n;
    BC_HIP_TRY(hipMalloc((void**)&g.row_ptr, sizeof(uint32_t) * (n + 1)));
    BC_HIP_TRY(hipMalloc((void**)&g.csc_ptr, sizeof(uint32_t) * (n + 1)));
    BC_HIP_TRY(hipMemsetAsync(g.row_ptr, 0, sizeof(uint32_t) * (n + 1), st));
    BC_HIP_TRY(hipMemsetAsync(g.csc_ptr, 0, sizeof(uint32_t) * (n + 1), st));

    uint32_t* counters = nullptr;   // [0] kept pairs, [1] bad id, [2] unique edges, [3] max degree
    BC_HIP_TRY(hipMallocAsync((void**)&counters, 4 * sizeof(uint32_t), st));
    BC_HIP_TRY(hipMemsetAsync(counters, 0, 4 * sizeof(uint32_t), st));
    uint32_t h[4] = {0, 0, 0, 0};

    uint64_t *keys = nullptr, *tmp = nullptr;
    if (M > 0) {
        BC_HIP_TRY(hipMallocAsync((void**)&keys, M * sizeof(uint64_t), st));
        BC_HIP_TRY(hipMallocAsync((void**)&tmp, M * sizeof(uint64_t), st));
        hipLaunchKernelGGL(k_pack, dim3(grid_for(M, 256)), dim3(256), 0, st, d_src, d_dst, M, (uint32_t)n, vbits,
                           keys, counters);
        BC_HIP_TRY(hipGetLastError());
        BC_HIP_TRY(hipMemcpyAsync(h, counters, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipStreamSynchronize(st));
    }
    if (h[1]) {
        (void)hipFreeAsync(keys, st);
        (void)hipFreeAsync(tmp, st);
        (void)hipFreeAsync(counters, st);
        (void)hipStreamSynchronize(st);
        throw Error{BC_E_RANGE, "edge list holds a vertex id >= n"};
    }
    const uint64_t K = h[0];
    uint32_t m = 0;
    if (K > 0) {
        uint64_t* sorted = radix_sort(keys, tmp, K, 2 * vbits, st);
        uint64_t* other = (sorted == keys) ? tmp : keys;
        uint32_t *flags = nullptr, *pos = nullptr;
        BC_HIP_TRY(hipMallocAsync((void**)&flags, K * sizeof(uint32_t), st));
        BC_HIP_TRY(hipMallocAsync((void**)&pos, K * sizeof(uint32_t), st));
        hipLaunchKernelGGL(k_first_flags, dim3(grid_for(K, 256)), dim3(256), 0, st, sorted, K, flags);
        BC_HIP_TRY(hipGetLastError());
        scan_u32(flags, pos, K, st);
        uint32_t last[2];
        BC_HIP_TRY(hipMemcpyAsync(&last[0], pos + K - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipMemcpyAsync(&last[1], flags + K - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        BC_HIP_TRY(hipStreamSynchronize(st));
        m = last[0] + last[1];
        BC_HIP_TRY(hipMalloc((void**)&g.col, sizeof(uint32_t) * std::max<uint32_t>(m, 1)));
        BC_HIP_TRY(hipMalloc((void**)&g.csc_row, sizeof(uint32_t) * std::max<uint32_t>(m, 1)));
        // out-degrees are counted into row_ptr[0..n), then scanned in place (row_ptr[n] = 0
        // before the scan, m after it)
        hipLaunchKernelGGL(k_unique_scatter, dim3(grid_for(K, 256)), dim3(256), 0, st, sorted, K, flags, pos, vbits,
                           other, g.col, g.row_ptr);
        BC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_max_u32, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0, st, g.row_ptr,
                           (uint64_t)n, counters + 3);
        BC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_count_zero, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0, st, g.row_ptr,
                           (uint64_t)n, counters + 1);
        BC_HIP_TRY(hipGetLastError());
        scan_u32(g.row_ptr, g.row_ptr, (uint64_t)n + 1, st);
        // CSC: sort the transposed keys of the unique edges
        uint64_t* tsorted = radix_sort(other, sorted, m, 2 * vbits, st);
        hipLaunchKernelGGL(k_csc_fill, dim3(grid_for(m, 256)), dim3(256), 0, st, tsorted, (uint64_t)m, vbits,
                           g.csc_row, g.csc_ptr);
        BC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_max_u32, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0, st, g.csc_ptr,
                           (uint64_t)n, counters + 2);
        BC_HIP_TRY(hipGetLastError());
        scan_u32(g.csc_ptr, g.csc_ptr, (uint64_t)n + 1, st);
        BC_HIP_TRY(hipFreeAsync(flags, st));
        BC_HIP_TRY(hipFreeAsync(pos, st));
        BC_HIP_TRY(hipMemcpyAsync(&h[1], counters + 1, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    } else {
        h[1] = (uint32_t)n;   // every vertex has out-degree 0
        h[2] = 0;
        BC_HIP_TRY(hipMalloc((void**)&g.col, sizeof(uint32_t)));
        BC_HIP_TRY(hipMalloc((void**)&g.csc_row, sizeof(uint32_t)));
    }
    const char* rl = std::getenv("BCMI_RELABEL");
    if (m > 0 && n >= kRelabelMinN && !(rl && rl[0] == '0')) {
        // kernel copy of the graph, vertices renumbered by decreasing in-degree (ties by id)
        BC_HIP_TRY(hipStreamSynchronize(st));
        const uint32_t maxin = h[2];
        int dbits = 1;
        while (dbits < 32 && (1ull << dbits) <= maxin) ++dbits;
        uint64_t *dk = nullptr, *dt = nullptr;
        BC_HIP_TRY(hipMallocAsync((void**)&dk, (size_t)n * 8, st));
        BC_HIP_TRY(hipMallocAsync((void**)&dt, (size_t)n * 8, st));
        BC_HIP_TRY(hipMalloc((void**)&g.perm, sizeof(uint32_t) * n));
        BC_HIP_TRY(hipMalloc((void**)&g.iperm, sizeof(uint32_t) * n));
        BC_HIP_TRY(hipMalloc((void**)&g.prow, sizeof(uint32_t) * (n + 1)));
        BC_HIP_TRY(hipMalloc((void**)&g.pcol, sizeof(uint32_t) * m));
        const unsigned gn = std::min<unsigned>(grid_for(n, 256), 4096);
        hipLaunchKernelGGL(k_degree_keys, dim3(gn), dim3(256), 0, st, g.csc_ptr, (uint32_t)n, maxin, vbits, dk);
        BC_HIP_TRY(hipGetLastError());
        uint64_t* ds = radix_sort(dk, dt, (uint64_t)n, dbits + vbits, st);
        hipLaunchKernelGGL(k_perm_from_sorted, dim3(gn), dim3(256), 0, st, ds, (uint32_t)n, vbits, g.iperm, g.perm);
        BC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_relabel_keys, dim3(gn), dim3(256), 0, st, g.row_ptr, g.col, (uint32_t)n, g.perm, vbits,
                           keys);
        BC_HIP_TRY(hipGetLastError());
        uint64_t* rs = radix_sort(keys, tmp, m, 2 * vbits, st);
        BC_HIP_TRY(hipMemsetAsync(g.prow, 0, sizeof(uint32_t) * (n + 1), st));
        hipLaunchKernelGGL(k_csr_from_sorted, dim3(std::min<unsigned>(grid_for(m, 256), 8192)), dim3(256), 0, st, rs,
                           (uint64_t)m, vbits, g.pcol);
        BC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_relabel_degrees, dim3(gn), dim3(256), 0, st, g.row_ptr, g.iperm, (uint32_t)n, g.prow);
        BC_HIP_TRY(hipGetLastError());
        scan_u32(g.prow, g.prow, (uint64_t)n + 1, st);
        BC_HIP_TRY(hipFreeAsync(dk, st));
        BC_HIP_TRY(hipFreeAsync(dt, st));
    }
    if (keys) BC_HIP_TRY(hipFreeAsync(keys, st));
    if (tmp) BC_HIP_TRY(hipFreeAsync(tmp, st));
    BC_HIP_TRY(hipFreeAsync(counters, st));
    BC_HIP_TRY(hipStreamSynchronize(st));
    g.m = m;
    g.max_out_degree = h[3];
    g.max_in_degree = h[2];
    g.zero_out_degree = h[1];
    build_order(g, vbits, st);
    BC_HIP_TRY(hipStreamSynchronize(st));
}

}  // namespace bcmi
