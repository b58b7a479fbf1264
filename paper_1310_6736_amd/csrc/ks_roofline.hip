// Roofline microbenchmarks: the ceilings the search kernels are measured against.
//   KS_ROOF_COPY        streaming copy (read + write) over a large device buffer
//   KS_ROOF_LDS_ADD64   conflict-free 64-bit LDS atomic adds (each lane its own
//                       address, consecutive lanes in consecutive banks)
//   KS_ROOF_LDS_ADD32   conflict-free 32-bit LDS atomic adds
//   KS_ROOF_LDS_ADD64_SHARED4  64-bit LDS adds, 4 lanes per address (16 replicas
//                       per wavefront, as in the mean-shift scatter), all lanes
//                       of a replica hitting the same bin: the worst case
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ks.h"

namespace ks {

constexpr int kLdsWords = 2048;  // 16 KB of u64 per workgroup
constexpr int kIters = 4096;

__global__ __launch_bounds__(256) void k_lds_add64(unsigned long long* sink, int shared4) {
    __shared__ unsigned long long h[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += 256) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = shared4 ? (lane & 15) : lane;
    unsigned long long* base = h + wave * 512 + slot;
    unsigned long long inc = 1 + threadIdx.x;
#pragma unroll 16
    for (int i = 0; i < kIters; ++i) {
        atomicAdd(base + ((i & 7) << 6), inc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kLdsWords; i += 97) s += h[i];
        atomicAdd(sink, s);
    }
}

__global__ __launch_bounds__(256) void k_lds_add32(unsigned long long* sink) {
    __shared__ uint32_t h[kLdsWords * 2];
    for (int i = threadIdx.x; i < kLdsWords * 2; i += 256) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t* base = h + wave * 1024 + lane;
    const uint32_t inc = 1 + threadIdx.x;
#pragma unroll 16
    for (int i = 0; i < kIters; ++i) {
        atomicAdd(base + ((i & 7) << 6), inc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kLdsWords * 2; i += 97) s += h[i];
        atomicAdd(sink, s);
    }
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ a, uint4* __restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

}  // namespace ks

extern "C" {

// Runs one microbenchmark on `device` and returns its rate: bytes/s (copy: read +
// written) or lane-level LDS atomic operations per second.
ks_status ks_roofline(int32_t device, int32_t kind, double* rate) {
    if (!rate || kind < KS_ROOF_COPY || kind > KS_ROOF_LDS_ADD64_SHARED4) return KS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return KS_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return KS_E_DEVICE;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KS_E_DEVICE;
    ks_status st = KS_OK;
    float best_ms = 1e30f;
    if (kind == KS_ROOF_COPY) {
        const size_t bytes = (size_t)1 << 30;  // 1 GiB each way, far beyond the caches
        void *a = nullptr, *b = nullptr;
        if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
            st = KS_E_NOMEM;
        } else {
            hipMemset(a, 1, bytes);
            const size_t n = bytes / sizeof(uint4);
            const int grid = prop.multiProcessorCount * 8;
            for (int r = 0; r < 6 && st == KS_OK; ++r) {
                hipEventRecord(e0, 0);
                hipLaunchKernelGGL(ks::k_copy, dim3(grid), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
                hipEventRecord(e1, 0);
                if (hipEventSynchronize(e1) != hipSuccess) st = KS_E_DEVICE;
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (r > 0 && ms < best_ms) best_ms = ms;
            }
            if (st == KS_OK) *rate = 2.0 * (double)bytes / (best_ms * 1e-3);
        }
        if (a) hipFree(a);
        if (b) hipFree(b);
    } else {
        unsigned long long* sink = nullptr;
        if (hipMalloc(&sink, sizeof(unsigned long long)) != hipSuccess) {
            st = KS_E_NOMEM;
        } else {
            const int grid = prop.multiProcessorCount * 8;
            for (int r = 0; r < 6 && st == KS_OK; ++r) {
                hipEventRecord(e0, 0);
                if (kind == KS_ROOF_LDS_ADD32)
                    hipLaunchKernelGGL(ks::k_lds_add32, dim3(grid), dim3(256), 0, 0, sink);
                else
                    hipLaunchKernelGGL(ks::k_lds_add64, dim3(grid), dim3(256), 0, 0, sink,
                                       kind == KS_ROOF_LDS_ADD64_SHARED4 ? 1 : 0);
                hipEventRecord(e1, 0);
                if (hipEventSynchronize(e1) != hipSuccess) st = KS_E_DEVICE;
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (r > 0 && ms < best_ms) best_ms = ms;
            }
            if (st == KS_OK) *rate = (double)grid * 256.0 * ks::kIters / (best_ms * 1e-3);
            hipFree(sink);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return st;
}

}  // extern "C"
