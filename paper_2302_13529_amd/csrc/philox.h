// philox.h -- Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
// as 1, 2, 3", SC'11) for the live-edge coins of the GPU kernels. The counter is
// (edge quad, sample index, 0, 0) for the independent cascade model's edge coins and
// (vertex quad, sample index, 1, 0) for the linear-threshold model's vertex choices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imin {

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1,
                                              uint32_t &r0, uint32_t &r1, uint32_t &r2,
                                              uint32_t &r3, uint32_t c2 = 0u)
{
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product in one multiply (v_mad_u64_u32), not a low and a
        // high multiply
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        x0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        x1 = (uint32_t)p1;
        x2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    r0 = x0;
    r1 = x1;
    r2 = x2;
    r3 = x3;
}

// Live-edge bits of one quad of 4 edges for sample j: bit i is set when edge 4*quad+i lies in
// [e0, e1) and its 24-bit coin falls under its threshold ceil(p * 2^24).
__device__ __forceinline__ uint32_t live_mask(int quad, uint32_t j, uint32_t key_lo,
                                              uint32_t key_hi, int e0, int e1, uint4 thr)
{
    uint32_t w0, w1, w2, w3;
    philox4x32_10((uint32_t)quad, j, key_lo, key_hi, w0, w1, w2, w3);
    const int eb = quad * 4;
    uint32_t mask = 0;
    mask |= (eb + 0 >= e0 && eb + 0 < e1 && (w0 >> 8) < thr.x) ? 1u : 0u;
    mask |= (eb + 1 >= e0 && eb + 1 < e1 && (w1 >> 8) < thr.y) ? 2u : 0u;
    mask |= (eb + 2 >= e0 && eb + 2 < e1 && (w2 >> 8) < thr.z) ? 4u : 0u;
    mask |= (eb + 3 >= e0 && eb + 3 < e1 && (w3 >> 8) < thr.w) ? 8u : 0u;
    return mask;
}

// Linear-threshold model (a triggering model, Section V-E): vertex u keeps the in-edge whose
// 24-bit interval [lo, hi) holds u's choice R = word (u & 3) of Philox4x32-10 at counter
// (u >> 2, j, 1, 0), shifted right by 8. Live bits of one quad whose targets are `col`.
__device__ __forceinline__ uint32_t vertex_choice(uint32_t u, uint32_t j, uint32_t key_lo,
                                                  uint32_t key_hi)
{
    uint32_t w0, w1, w2, w3;
    philox4x32_10(u >> 2, j, key_lo, key_hi, w0, w1, w2, w3, 1u);
    const uint32_t w = (u & 3) == 0 ? w0 : (u & 3) == 1 ? w1 : (u & 3) == 2 ? w2 : w3;
    return w >> 8;
}

__device__ __forceinline__ uint32_t live_mask_lt(int quad, uint32_t j, uint32_t key_lo,
                                                 uint32_t key_hi, int e0, int e1, uint4 lo,
                                                 uint4 hi, uint4 col)
{
    const int eb = quad * 4;
    uint32_t mask = 0;
    const uint32_t l[4] = {lo.x, lo.y, lo.z, lo.w};
    const uint32_t h[4] = {hi.x, hi.y, hi.z, hi.w};
    const uint32_t c[4] = {col.x, col.y, col.z, col.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (eb + i < e0 || eb + i >= e1 || h[i] == 0u) continue;  // out of row, or masked
        const uint32_t r = vertex_choice(c[i], j, key_lo, key_hi);
        if (r >= l[i] && r < h[i]) mask |= 1u << i;
    }
    return mask;
}

}  // namespace imin
