// Approximate BC by source sampling (the approximation the paper cites in section I): BC
// estimated from k pivot sources drawn uniformly with replacement, scaled by n/k, which is
// unbiased because BC(v) = sum over all s of delta_s(v).
//
//   * bc_approx: k from a Hoeffding bound.  Each term n * delta_s(v) lies in [0, n(n-2)], so
//     with k >= ln(2n/delta) / (2 eps^2) pivots every vertex's estimate is within
//     eps * n(n-2) of BC(v) with probability at least 1 - delta (union bound over the n
//     vertices).  When that k reaches n the exact BC is computed instead.
//   * bc_approx_vertex: adaptive sampling for one vertex v (stop once the sampled
//     dependencies of v reach c * n, estimate n * S / k), in rounds of 64 pivots.
//
// Pivots come from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014), mapped to [0, n) by a 64x64->128-bit multiply.  All sampling runs
// on the host; the dependencies come from the sampled-BC kernels.
#include "bc_internal.h"

#include <cmath>
#include <vector>

namespace bcmi {

namespace {

__global__ void k_scale(double* bc, uint32_t n, double f) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) bc[v] *= f;
}

__global__ void k_pick(const double* bc, uint32_t v, double* out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = bc[v];
}

uint64_t splitmix64_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

void draw_pivots(uint64_t seed, uint32_t n, uint32_t k, uint32_t* out) {
    uint64_t state = seed;
    for (uint32_t i = 0; i < k; ++i)
        out[i] = (uint32_t)(((unsigned __int128)splitmix64_next(state) * n) >> 64);
}

uint32_t hoeffding_pivots(uint32_t n, double eps, double delta) {
    BC_REQUIRE(eps > 0.0 && eps <= 1.0, BC_E_INVAL, "eps must be in (0, 1]");
    BC_REQUIRE(delta > 0.0 && delta < 1.0, BC_E_INVAL, "delta must be in (0, 1)");
    const double k = std::ceil(std::log(2.0 * std::max<uint32_t>(n, 1) / delta) / (2.0 * eps * eps));
    return k >= (double)n ? n : (uint32_t)k;
}

void scale_bc(double* d_bc, uint32_t n, double f, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(std::max(1u, std::min((n + 255) / 256, 4096u))), dim3(256), 0, st, d_bc, n, f);
    BC_HIP_TRY(hipGetLastError());
}

double read_bc_entry(const double* d_bc, uint32_t v, double* d_tmp, hipStream_t st) {
    hipLaunchKernelGGL(k_pick, dim3(1), dim3(64), 0, st, d_bc, v, d_tmp);
    BC_HIP_TRY(hipGetLastError());
    double h = 0.0;
    BC_HIP_TRY(hipMemcpyAsync(&h, d_tmp, sizeof(double), hipMemcpyDeviceToHost, st));
    BC_HIP_TRY(hipStreamSynchronize(st));
    return h;
}

}  // namespace bcmi
