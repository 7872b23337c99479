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
            // hi ^ c ^ k as one three-input bit operation (truth table 0x96:
            // the parity of the three inputs); the compiler issues two xors
            const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
            const uint32_t n1 = (uint32_t)pb;
            const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
            const uint32_t n3 = (uint32_t)pa;
            c0 = n0; c1 = n1; c2 = n2; c3 = n3;
            k0 += kWeylA;
            k1 += kWeylB;
        }
        return Out{c0, c1, c2, c3};
    }
};

// Index of workgroup b of n such that workgroups on one XCD get consecutive
// indices.  The dispatcher deals workgroups to the 8 XCDs in turn, so b,
// b + 8, b + 16, ... share an XCD and its L2; they map to one run of
// consecutive indices (the first n mod 8 XCDs take one more than the
// others).  A bijection of [0, n): neighbouring trajectories of a
// trajectory-minor array then share cache lines within one L2.
__device__ __forceinline__ int64_t xcd_local_index(int64_t b, int64_t n)
{
    constexpr int64_t kXcd = 8;
    const int64_t base = n / kXcd, rem = n % kXcd, x = b % kXcd;
    return x * base + (x < rem ? x : rem) + b / kXcd;
}

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

// --------------------------------------------------------------------------
// Reductions over aligned groups of L lanes (L = 8, 16, 32, 64) without LDS:
// DPP lane permutations inside rows of 16 lanes (pairs at xor 1 and 2, then
// mirrors of 8 and 16 lanes) and the gfx950 row swaps across rows and halves.
// Each step combines a lane's value with its partner's by a commutative
// operation, so every lane of a group ends with bitwise the same result.
// All lanes of the wavefront must be active.
namespace lanes {

constexpr int kXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141;
constexpr int kMirror = 0x140;
constexpr int kRowBcast0 = 0x150;  // lane 0 of each row
constexpr int kRowBcast8 = 0x158;  // lane 8 of each row

template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    // every control used here reads a valid lane, so bound_ctrl only spares
    // the copy of the old value
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp<CTRL>(__float_as_int(v)));
}

// (value of the even row, value of the odd row) of each pair of rows
__device__ __forceinline__ void rows16(int v, int &even, int &odd)
{
    const auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    even = (int)p[0];
    odd = (int)p[1];
}

// (value of the lower half, value of the upper half)
__device__ __forceinline__ void halves(int v, int &lo, int &hi)
{
    const auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    lo = (int)p[0];
    hi = (int)p[1];
}

__device__ __forceinline__ void rows16(float v, float &even, float &odd)
{
    int e, o;
    rows16(__float_as_int(v), e, o);
    even = __int_as_float(e);
    odd = __int_as_float(o);
}

__device__ __forceinline__ void halves(float v, float &lo, float &hi)
{
    int a, b;
    halves(__float_as_int(v), a, b);
    lo = __int_as_float(a);
    hi = __int_as_float(b);
}

}  // namespace lanes

template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(L == 8 || L == 16 || L == 32 || L == 64, "group width");
    v += lanes::dpp<lanes::kXor1>(v);
    v += lanes::dpp<lanes::kXor2>(v);
    v += lanes::dpp<lanes::kHalfMirror>(v);
    if (L >= 16) v += lanes::dpp<lanes::kMirror>(v);
    if (L >= 32) {
        float e, o;
        lanes::rows16(v, e, o);
        v = e + o;
    }
    if (L >= 64) {
        float lo, hi;
        lanes::halves(v, lo, hi);
        v = lo + hi;
    }
    return v;
}

template <int L>
__device__ __forceinline__ float group_min(float v)
{
    static_assert(L == 8 || L == 16 || L == 32 || L == 64, "group width");
    v = fminf(v, lanes::dpp<lanes::kXor1>(v));
    v = fminf(v, lanes::dpp<lanes::kXor2>(v));
    v = fminf(v, lanes::dpp<lanes::kHalfMirror>(v));
    if (L >= 16) v = fminf(v, lanes::dpp<lanes::kMirror>(v));
    if (L >= 32) {
        float e, o;
        lanes::rows16(v, e, o);
        v = fminf(e, o);
    }
    if (L >= 64) {
        float lo, hi;
        lanes::halves(v, lo, hi);
        v = fminf(lo, hi);
    }
    return v;
}

// Race state (smallest ratio r1, its channel j1, second smallest r2) over a
// group of lanes.  Ratios are non-negative, so the bit pattern of r1 (with
// -0 made +0) orders like the value, and (r1, j1) packs into one 64-bit key
// whose unsigned minimum is the smaller ratio with the lowest channel on
// exact ties.  r2 is the smallest of the rest: min(a2, b2, max(a1, b1)).
namespace racekey {

__device__ __forceinline__ uint64_t pack(float r1, int j1)
{
    const uint32_t bits = (uint32_t)__float_as_int(r1 + 0.0f);
    return ((uint64_t)bits << 32) | (uint32_t)j1;
}

__device__ __forceinline__ float ratio(uint64_t k) { return __int_as_float((int)(uint32_t)(k >> 32)); }

__device__ __forceinline__ void merge(uint64_t &k, float &r2, uint64_t ko, float o2)
{
    r2 = fminf(fminf(r2, o2), fmaxf(ratio(k), ratio(ko)));
    k = ko < k ? ko : k;
}

template <int CTRL>
__device__ __forceinline__ void step(uint64_t &k, float &r2)
{
    const int lo = lanes::dpp<CTRL>((int)(uint32_t)k);
    const int hi = lanes::dpp<CTRL>((int)(uint32_t)(k >> 32));
    merge(k, r2, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo, lanes::dpp<CTRL>(r2));
}

}  // namespace racekey

template <int L>
__device__ __forceinline__ void group_race(float &r1, int &j1, float &r2)
{
    static_assert(L == 8 || L == 16 || L == 32 || L == 64, "group width");
    uint64_t k = racekey::pack(r1, j1);
    racekey::step<lanes::kXor1>(k, r2);
    racekey::step<lanes::kXor2>(k, r2);
    racekey::step<lanes::kHalfMirror>(k, r2);
    if (L >= 16) racekey::step<lanes::kMirror>(k, r2);
    if (L >= 32) {
        int elo, olo, ehi, ohi;
        float e2, o2;
        lanes::rows16((int)(uint32_t)k, elo, olo);
        lanes::rows16((int)(uint32_t)(k >> 32), ehi, ohi);
        lanes::rows16(r2, e2, o2);
        k = ((uint64_t)(uint32_t)ehi << 32) | (uint32_t)elo;
        r2 = e2;
        racekey::merge(k, r2, ((uint64_t)(uint32_t)ohi << 32) | (uint32_t)olo, o2);
    }
    if (L >= 64) {
        int llo, hlo, lhi, hhi;
        float l2, h2;
        lanes::halves((int)(uint32_t)k, llo, hlo);
        lanes::halves((int)(uint32_t)(k >> 32), lhi, hhi);
        lanes::halves(r2, l2, h2);
        k = ((uint64_t)(uint32_t)lhi << 32) | (uint32_t)llo;
        r2 = l2;
        racekey::merge(k, r2, ((uint64_t)(uint32_t)hhi << 32) | (uint32_t)hlo, h2);
    }
    r1 = racekey::ratio(k);
    j1 = (int)(uint32_t)k;
}

// Gumbel-Softmax temperature of a run: the device scalar when one is given.
template <class P>
__device__ __forceinline__ float run_temperature(const P &p)
{
    return p.d_temperature ? *p.d_temperature : p.temperature;
}

// The value of the first lane of each group.
template <int L>
__device__ __forceinline__ float group_first(float v)
{
    static_assert(L == 8 || L == 16 || L == 32 || L == 64, "group width");
    if (L == 64) return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    const float b0 = lanes::dpp<lanes::kRowBcast0>(v);
    if (L == 16) return b0;
    if (L == 32) {
        float e, o;
        lanes::rows16(b0, e, o);
        return e;
    }
    const float b8 = lanes::dpp<lanes::kRowBcast8>(v);
    return (__lane_id() & 8) ? b8 : b0;
}

}  // namespace ssa
