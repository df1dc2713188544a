// Achievable HBM bandwidth on this device, measured with STREAM-style kernels (copy b = a and
// triad a = b + q c over arrays far larger than the 256 MB MALL), so that a kernel's achieved
// bandwidth can be set against what plain streaming reaches on the same GPU, not only against
// the data-sheet peak.  Measurement utility only; no part of the betweenness computation.
#include "bc_internal.h"

#include <algorithm>
#include <vector>

namespace bcmi {

namespace {

constexpr int kProbeWG = 256;
constexpr int kProbeUnroll = 4;   // 16-byte elements per thread and pass, all loads before the stores

__global__ void __launch_bounds__(kProbeWG) k_probe_copy(const uint4* __restrict__ a, uint4* __restrict__ b,
                                                         size_t n16) {
    const size_t step = (size_t)gridDim.x * kProbeWG * kProbeUnroll;
    for (size_t base = (size_t)blockIdx.x * kProbeWG * kProbeUnroll + threadIdx.x; base < n16; base += step) {
        uint4 x[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + (size_t)u * kProbeWG;
            if (i < n16) x[u] = a[i];
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + (size_t)u * kProbeWG;
            if (i < n16) b[i] = x[u];
        }
    }
}

__global__ void __launch_bounds__(kProbeWG) k_probe_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                                          const double2* __restrict__ c, double q, size_t n16) {
    const size_t step = (size_t)gridDim.x * kProbeWG * kProbeUnroll;
    for (size_t base = (size_t)blockIdx.x * kProbeWG * kProbeUnroll + threadIdx.x; base < n16; base += step) {
        double2 x[kProbeUnroll], y[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + (size_t)u * kProbeWG;
            if (i < n16) {
                x[u] = b[i];
                y[u] = c[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + (size_t)u * kProbeWG;
            if (i < n16) a[i] = make_double2(x[u].x + q * y[u].x, x[u].y + q * y[u].y);
        }
    }
}

__global__ void k_probe_fill(double2* p, size_t n16, double v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_double2(v, v);
}

double median(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    const size_t h = v.size() / 2;
    return v.size() % 2 ? v[h] : 0.5 * ((double)v[h - 1] + v[h]);
}

}  // namespace

void stream_probe(size_t bytes, int reps, double* copy_gbs, double* triad_gbs) {
    const size_t n16 = bytes / 16;
    BC_REQUIRE(n16 >= 1, BC_E_INVAL, "array size below 16 bytes");
    BC_REQUIRE(reps >= 1, BC_E_INVAL, "reps must be >= 1");
    int dev = 0;
    BC_HIP_TRY(hipGetDevice(&dev));
    const DevInfo& di = dev_info(dev);
    const unsigned grid = (unsigned)std::max<size_t>(
        1, std::min<size_t>((size_t)di.cus * 8, (n16 + kProbeWG * kProbeUnroll - 1) / (kProbeWG * kProbeUnroll)));
    void* a = nullptr;
    void* b = nullptr;
    void* c = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&] {
        if (st) (void)hipStreamSynchronize(st);
        for (void* p : {a, b, c})
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    };
    try {
        BC_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        BC_HIP_TRY(hipEventCreate(&e0));
        BC_HIP_TRY(hipEventCreate(&e1));
        BC_HIP_TRY(hipMalloc(&a, n16 * 16));
        BC_HIP_TRY(hipMalloc(&b, n16 * 16));
        BC_HIP_TRY(hipMalloc(&c, n16 * 16));
        for (void* p : {a, b, c})
            hipLaunchKernelGGL(k_probe_fill, dim3(grid), dim3(kProbeWG), 0, st, (double2*)p, n16, 1.0);
        BC_HIP_TRY(hipGetLastError());
        std::vector<float> tc, tt;
        for (int r = 0; r <= reps; ++r) {   // the first pass of each kernel is a warm-up
            float ms = 0.f;
            BC_HIP_TRY(hipEventRecord(e0, st));
            hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kProbeWG), 0, st, (const uint4*)a, (uint4*)b, n16);
            BC_HIP_TRY(hipEventRecord(e1, st));
            BC_HIP_TRY(hipEventSynchronize(e1));
            BC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (r) tc.push_back(ms);
            BC_HIP_TRY(hipEventRecord(e0, st));
            hipLaunchKernelGGL(k_probe_triad, dim3(grid), dim3(kProbeWG), 0, st, (double2*)a, (const double2*)b,
                               (const double2*)c, 0.5, n16);
            BC_HIP_TRY(hipEventRecord(e1, st));
            BC_HIP_TRY(hipEventSynchronize(e1));
            BC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (r) tt.push_back(ms);
        }
        BC_HIP_TRY(hipGetLastError());
        const double bytes16 = (double)n16 * 16.0;
        if (copy_gbs) *copy_gbs = 2.0 * bytes16 / (median(tc) * 1e-3) / 1e9;
        if (triad_gbs) *triad_gbs = 3.0 * bytes16 / (median(tt) * 1e-3) / 1e9;
    } catch (...) {
        release();
        throw;
    }
    release();
}

}  // namespace bcmi
