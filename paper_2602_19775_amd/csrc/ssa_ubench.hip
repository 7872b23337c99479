// Instruction-throughput probes for the roofline of the SSA kernels: each
// kernel runs 8 independent dependency chains of one instruction kind per
// lane, at full occupancy, so the measured rate is the issue limit of that
// instruction kind on the vector ALU.  Separate library (libssa_ubench.so);
// the simulation library does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void probe(int iters, uint32_t seed, uint32_t *sink)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t u[kChains];
    float f[kChains];
    double d[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        u[c] = seed ^ (t * 0x9E3779B9u + c);
        f[c] = 1.5f + (float)((t + c) & 7);
        d[c] = 1.5 + (double)((t + c) & 7);
    }
    const uint32_t mul = 0xD2511F53u ^ seed;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (KIND == 0) {          // 32x32 -> 64-bit product (Philox multiply)
                const uint64_t p = (uint64_t)mul * u[c];
                u[c] = (uint32_t)(p >> 32) + (uint32_t)p;
            } else if (KIND == 1) {   // base-2 logarithm
                f[c] = __builtin_amdgcn_logf(f[c]) + 2.0f;
            } else if (KIND == 2) {   // reciprocal
                f[c] = __builtin_amdgcn_rcpf(f[c]) + 1.5f;
            } else if (KIND == 3) {   // FP32 fused multiply-add
                f[c] = __builtin_fmaf(f[c], 0.999f, 0.25f);
            } else if (KIND == 4) {   // 32-bit logic
                u[c] = (u[c] ^ mul) + 0x3C6EF372u;
            } else if (KIND == 5) {   // FP64 fused multiply-add
                d[c] = __builtin_fma(d[c], 0.999, 0.25);
            } else if (KIND == 6) {   // int -> float conversion
                f[c] = (float)(__float_as_uint(f[c]) >> 9);
            } else if (KIND == 7) {   // three-input bit operation (Philox's hi ^ c ^ k)
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], mul, 0x3C6EF372u, 0x96) + 0x3C6EF372u;
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= u[c] ^ __float_as_uint(f[c]) ^ (uint32_t)__double_as_longlong(d[c]);
    if (acc == 0x12345678u) sink[t] = acc;   // keeps the chains alive
}

}  // namespace

// ops per lane executed by probe kind `kind` with `iters` iterations
extern "C" double ubench_ops_per_lane(int kind, int iters)
{
    // kinds 0, 1, 2, 4, 6 and 7 issue two instructions per chain step
    const double per = (kind == 3 || kind == 5) ? 1.0 : 2.0;
    return per * kChains * (double)iters;
}

// Runs probe `kind` on `blocks` x 256 lanes; returns the kernel time in ms (<0 on error).
extern "C" float ubench_run(int kind, int iters, int blocks)
{
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, sizeof(uint32_t) * (size_t)blocks * 256) != hipSuccess) return -1.f;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto launch = [&](void) {
        switch (kind) {
        case 0: hipLaunchKernelGGL(probe<0>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 1: hipLaunchKernelGGL(probe<1>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 2: hipLaunchKernelGGL(probe<2>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 3: hipLaunchKernelGGL(probe<3>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 4: hipLaunchKernelGGL(probe<4>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 5: hipLaunchKernelGGL(probe<5>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        case 6: hipLaunchKernelGGL(probe<6>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        default: hipLaunchKernelGGL(probe<7>, dim3(blocks), dim3(256), 0, 0, iters, 7u, sink); break;
        }
    };
    launch();   // warm-up
    (void)hipEventRecord(e0, 0);
    launch();
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = -1.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return ms;
}
