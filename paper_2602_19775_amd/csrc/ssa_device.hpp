// Device primitives of the SSA kernels (gfx950): the Philox4x32-10 counter
// stream, the uniform lattice and -ln(u), and the packed channel tables.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "ssa_plan.hpp"

#ifndef INFINITY
#define INFINITY __builtin_inff()
#endif

namespace ssa {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplies with the Weyl key schedule.  The key is wave-uniform (the seed),
// so the schedule lives in scalar registers; counter words that are uniform
// (block, step, purpose/epoch) keep the first rounds partly scalar.
struct Philox {
    static constexpr uint32_t kMulA = 0xD2511F53u;
    static constexpr uint32_t kMulB = 0xCD9E8D57u;
    static constexpr uint32_t kWeylA = 0x9E3779B9u;
    static constexpr uint32_t kWeylB = 0xBB67AE85u;

    struct Out {
        uint32_t x, y, z, w;
    };

    __device__ __forceinline__ static Out block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
    {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t pa = (uint64_t)kMulA * c0;
            const uint64_t pb = (uint64_t)kMulB * c2;
            const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
            const uint32_t n1 = (uint32_t)pb;
            const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
            const uint32_t n3 = (uint32_t)pa;
            c0 = n0; c1 = n1; c2 = n2; c3 = n3;
            k0 += kWeylA;
            k1 += kWeylB;
        }
        return Out{c0, c1, c2, c3};
    }
};

// Lattice uniform u = (2*(x>>9)+1) * 2^-24, exact in FP32 and strictly inside (0,1).
__device__ __forceinline__ float lattice_u(uint32_t x)
{
    return (float)((x >> 8) | 1u) * 0x1p-24f;
}

// E = -ln(u) in FP32 for a lattice word.  The lattice excludes 0 and 1 and
// never reaches the denormal range, so the hardware base-2 logarithm needs no
// range scaling: E = -log2(u) * ln 2.  Its relative error over all 2^23
// lattice points is checked exhaustively against FP64 by the self-test entry
// point.
__device__ __forceinline__ float neglog_u(uint32_t x)
{
    return __builtin_amdgcn_logf(lattice_u(x)) * -0.693147180559945309f;
}

// Signed 4-bit field s of a packed change-vector word.
__device__ __forceinline__ int nibble(uint32_t w, int s)
{
    return ((int)(w << (28 - 4 * s))) >> 28;
}

__device__ __forceinline__ float fast_rcp(float x)
{
    return __builtin_amdgcn_rcpf(x);
}

// Wave-uniform broadcast of a value every active lane agrees on.
__device__ __forceinline__ int uniform_i(int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

// Lanes of the wavefront whose predicate holds (the compare mask itself).
__device__ __forceinline__ uint64_t ballot(bool p)
{
    return __builtin_amdgcn_ballot_w64(p);
}

}  // namespace ssa
