// Memory-system rate probe (not part of the library): 1024-thread
// workgroups issue 64-bit atomic minima, or plain loads, at pseudo-random
// addresses of a 32 MiB buffer (beyond an XCD's L2) or a 2 MiB one (inside
// it), eight in flight per lane.  It gives the ceilings the weighted
// searches' relaxations and the BFS's mask gathers run against: per-CU issue
// rate with one workgroup, and the device-wide rate with 64 and 256.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

enum { kAtomicWg = 0, kAtomicAgent = 1, kLoad = 2 };

template <int MODE>
__global__ __launch_bounds__(1024) void k_probe(uint64_t* buf, uint32_t mask, int iters, uint64_t* sink) {
    uint32_t x = 2654435761u * (threadIdx.x + 1) + blockIdx.x * 97u;
    uint64_t acc = 0;
    for (int i = 0; i < iters; i++) {
        uint64_t r[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            x ^= x << 13;
            x ^= x >> 17;
            x ^= x << 5;
            const uint32_t idx = x & mask;  // mask = size - 1: always in bounds
            if (MODE == kAtomicWg)
                r[q] = __hip_atomic_fetch_min(&buf[idx], (uint64_t)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else if (MODE == kAtomicAgent)
                r[q] = __hip_atomic_fetch_min(&buf[idx], (uint64_t)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                r[q] = buf[idx];
        }
#pragma unroll
        for (int q = 0; q < 8; q++) acc += r[q];
    }
    if (acc == 12345) sink[0] = 1;  // keeps the results live
}

template <int MODE>
void run(const char* name, int blocks, uint32_t size) {
    uint64_t *buf = nullptr, *sink = nullptr;
    CHECK(hipMalloc(&buf, sizeof(uint64_t) * size));
    CHECK(hipMemset(buf, 0xFF, sizeof(uint64_t) * size));
    CHECK(hipMalloc(&sink, 8));
    const int iters = 200;
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(1024), 0, 0, buf, size - 1, iters, sink);  // warm-up
    CHECK(hipEventRecord(a, 0));
    hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(1024), 0, 0, buf, size - 1, iters, sink);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    const double ops = (double)blocks * 1024 * iters * 8;
    std::printf("%-32s %3u MiB, workgroups=%3d: %8.3f ms, %6.2f G lane-ops/s, %6.2f cycles per lane-op per CU at 2.4 GHz\n",
                name, (unsigned)(size >> 17), blocks, ms, ops / ms / 1e6, (ms * 2.4e6) / (ops / blocks));
    CHECK(hipFree(buf));
    CHECK(hipFree(sink));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
}

int main() {
    for (uint32_t size : {1u << 22, 1u << 18}) {  // 32 MiB, 2 MiB of 64-bit words
        for (int blocks : {1, 64, 256}) {
            run<kAtomicWg>("atomic min u64, workgroup scope", blocks, size);
            run<kAtomicAgent>("atomic min u64, agent scope", blocks, size);
            run<kLoad>("load u64", blocks, size);
        }
    }
    return 0;
}
