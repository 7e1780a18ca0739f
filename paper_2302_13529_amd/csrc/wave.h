// wave.h -- wavefront-level helpers shared by the wave-sized kernels of libimin (small.hip,
// pack.hip): lane arithmetic, wave scans and sums, the seed-level register cache and the
// per-wave work counters.
#pragma once

#include "imin_internal.h"

namespace imin {
namespace wave {

constexpr int kSeedSlots = 4;                      // cached seed quads per lane
constexpr int kSeedCacheQuads = 64 * kSeedSlots;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Orders this wave's LDS accesses across lanes (the hardware runs one wave's LDS
// instructions in order; this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sum across the wave with data-parallel-primitive (DPP) lane moves, which
// stay in the vector unit: a log-step scan inside each row of 16 lanes (row_shr 1, 2, 4, 8),
// then the totals of rows 0 and 2 broadcast into rows 1 and 3 (row_bcast:15) and the total of
// rows 0-1 into rows 2 and 3 (row_bcast:31). Lanes without a source add the old value 0.
__device__ __forceinline__ int wave_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Sum over the wave, the same value in every lane (scalar register).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readlane(wave_scan((int)v), 63);
}

__device__ __forceinline__ int quads_of(int e0, int e1)
{
    return (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
}

__device__ __forceinline__ int pick(uint4 v, int i)
{
    return (int)(i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w);
}

// The current instance's seed level: quad p of the seed frontier sits in lane p % 64,
// slot p / 64. vmask holds the edges of the quad that belong to the seed's row.
struct SeedCache {
    int quad[kSeedSlots];
    uint4 thr[kSeedSlots];
    uint4 col[kSeedSlots];
    uint32_t vmask[kSeedSlots];
    int total;         // cached quads (uniform); -1 when the seed rows do not fit
    uint32_t scanned;  // out-edges of the seeds (uniform)
};

// e0, e1, ex: 64 ints of LDS scratch each, private to the calling wave.
__device__ inline void build_seed_cache(const InstanceDesc &I, int *e0s, int *e1s, int *exs,
                                        SeedCache &sc)
{
    const int lane = lane_id();
    int total = 0;
    uint32_t scanned = 0;
    for (int base = 0; base < I.nseeds; base += 64) {
        const int k = base + lane;
        int e0 = 0, e1 = 0;
        if (k < I.nseeds) {
            const int v = I.seeds[k];
            e0 = I.row_ptr[v];
            e1 = I.row_ptr[v + 1];
        }
        total += (int)wave_sum((uint32_t)quads_of(e0, e1));
        scanned += wave_sum((uint32_t)(e1 - e0));
    }
    sc.scanned = scanned;
#pragma unroll
    for (int s = 0; s < kSeedSlots; ++s) {
        sc.quad[s] = 0;
        sc.thr[s] = make_uint4(0, 0, 0, 0);
        sc.col[s] = make_uint4(0, 0, 0, 0);
        sc.vmask[s] = 0;
    }
    if (total > kSeedCacheQuads) {
        sc.total = -1;
        return;
    }
    sc.total = total;
    int off = 0;
    for (int base = 0; base < I.nseeds; base += 64) {
        const int k = base + lane;
        int e0 = 0, e1 = 0;
        if (k < I.nseeds) {
            const int v = I.seeds[k];
            e0 = I.row_ptr[v];
            e1 = I.row_ptr[v + 1];
        }
        const int nq = quads_of(e0, e1);
        const int incl = wave_scan(nq);
        const int ctot = __builtin_amdgcn_readlane(incl, 63);
        wave_sync();
        e0s[lane] = e0;
        e1s[lane] = e1;
        exs[lane] = incl - nq;
        wave_sync();
        const int cnt = min(64, I.nseeds - base);
#pragma unroll
        for (int s = 0; s < kSeedSlots; ++s) {
            const int q = lane + 64 * s - off;
            if (q >= 0 && q < ctot) {
                int l = 0, h = cnt - 1;
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (exs[mid] <= q) l = mid;
                    else h = mid - 1;
                }
                const int f0 = e0s[l], f1 = e1s[l];
                const int quad = (f0 >> 2) + (q - exs[l]);
                const int eb = quad * 4;
                uint32_t vm = 0;
                for (int i = 0; i < 4; ++i)
                    if (eb + i >= f0 && eb + i < f1) vm |= 1u << i;
                sc.quad[s] = quad;
                sc.vmask[s] = vm;
            }
        }
        off += ctot;
    }
#pragma unroll
    for (int s = 0; s < kSeedSlots; ++s) {
        if (sc.vmask[s]) {
            sc.thr[s] = I.thr4[sc.quad[s]];
            sc.col[s] = I.col4[sc.quad[s]];
        }
    }
}

// Work counters of the current instance, kept per wave and added to the instance's
// counters when the wave moves to another instance or ends.
struct Tally {
    unsigned long long samples, reached, scanned, live;
};

// pack: the samples were finished by the packed kernel (also counted there).
__device__ __forceinline__ void flush(const InstanceDesc &I, Tally &t, bool pack = false)
{
    if (t.samples == 0) return;
    if (lane_id() == 0) {
        atomicAdd(&I.stats[0], t.samples);
        atomicAdd(&I.stats[1], t.reached);
        atomicAdd(&I.stats[2], t.scanned);
        atomicAdd(&I.stats[3], t.live);
        atomicAdd(&I.stats[5], t.samples);
        if (pack) atomicAdd(&I.stats[6], t.samples);
    }
    t.samples = t.reached = t.scanned = t.live = 0;
}

}  // namespace wave
}  // namespace imin
