// small.hip -- Algorithm 2 of arXiv 2302.13529 for samples that stay small: one wavefront per
// sample, every per-sample array in LDS, no block barrier anywhere.
//
// Waves take samples, a few consecutive ones at a time, from a work counter spanning all
// instances of the launch, so many graphs (the batched form) or one graph share the same
// launch. Per sample:
//   * live edges are decided per 4-edge quad with the same Philox4x32-10 coin as the large
//     kernel (Definition 4; or the linear-threshold model's vertex choices, Section V-E);
//     lanes work on consecutive quads of the frontier;
//   * reachability from the merged seed is a wave-synchronous BFS. The live edges a wave
//     finds are claimed one at a time in lane order: the ids of the reached vertices are
//     mirrored in registers (4 per lane), so "already reached?" is one compare and a ballot;
//   * dominators use the same Jacobi NCA raising from the BFS tree as the large kernel, and
//     subtree sizes the same bottom-up pass over BFS levels (LDS atomics), with the sizes
//     added into the instance's 64-bit counters D (Algorithm 2, Theorem 6).
// Every sample of an instance expands the same seed rows, and only their coins differ; so a
// wave keeps the seed quads of its current instance in registers (thresholds and targets)
// and the seed level costs no memory traffic. Edges into seeds and blocked vertices have
// threshold 0 during a call, so no sample ever finds them live.
// A sample that reaches kSmallV - 1 vertices, keeps more than kSmallX extra edges, or meets a
// frontier chunk with more than the launch's quad limit is abandoned (nothing accumulated)
// and listed for the large kernel, so results never depend on which path ran.
#include "imin_internal.h"
#include "philox.h"
#include "wave.h"

namespace imin {
namespace {

using namespace wave;

constexpr int kSW = kSmallWaves;
constexpr int kSmallBlock = kSW * 64;
constexpr int kMaxSmallJacobiRounds = 4 * kSmallV;
constexpr uint32_t kPickMin = 4;                   // samples per work-counter update: a
constexpr uint32_t kPickMax = 64;                  // share of what remains, within these

struct WaveState {
    int gl[kSmallV];  // vertex id of each local id (local 0 is the merged seed: -1)
    int pa[kSmallV];  // parent in the BFS spanning tree
    int td[kSmallV];  // tentative immediate dominator
    int tn[kSmallV];  // next tentative dominator, then subtree sizes
    int lvl[kSmallV + 1];
    int2 extra[kSmallX];
    int e0[64], e1[64], ex[64];  // current 64-entry frontier chunk: edge range, quad prefix
};

struct SmallShared {
    WaveState w[kSW];
};

// Per-lane copy of the reached vertex ids: lane l holds local ids l, 64+l, 128+l, 192+l.
// Four named registers rather than an array: the compiler turns a write to row id >> 6 of an
// array into a store at a run-time index, which puts the whole array in scratch memory.
static_assert(kSmallV == 4 * 64, "the mirror holds four rows of 64 local ids");
struct Mirror {
    int g0 = -1, g1 = -1, g2 = -1, g3 = -1;
};

__device__ __forceinline__ void mirror_set(Mirror &m, int id, int v)
{
    const bool mine = lane_id() == (id & 63);
    const int r = id >> 6;
    m.g0 = (mine && r == 0) ? v : m.g0;
    m.g1 = (mine && r == 1) ? v : m.g1;
    m.g2 = (mine && r == 2) ? v : m.g2;
    m.g3 = (mine && r == 3) ? v : m.g3;
}

// Local id of vertex c (uniform across the wave), or -1.
__device__ __forceinline__ int mirror_find(const Mirror &m, int c)
{
    const int lane = lane_id();
    int hit = -1;
    hit = m.g0 == c ? lane : hit;
    hit = m.g1 == c ? 64 + lane : hit;
    hit = m.g2 == c ? 128 + lane : hit;
    hit = m.g3 == c ? 192 + lane : hit;
    const unsigned long long b = __ballot(hit >= 0);
    if (!b) return -1;
    return __builtin_amdgcn_readlane(hit, (int)__builtin_ctzll(b));
}

struct SampleCtx {
    int nV, nX, L;     // uniform
    int ovf;           // uniform
    int reach_only;    // uniform: keep no extra edges
    uint32_t live;     // per lane, summed at the end
    uint32_t scanned;  // per lane, summed at the end
};

// Claim live edge src -> c, whose target is known to be eligible (c, src uniform).
__device__ __forceinline__ void claim(WaveState &ws, Mirror &m, SampleCtx &cx, int c, int src)
{
    const int l = mirror_find(m, c);
    if (l < 0) {
        if (cx.nV >= kSmallV) {
            cx.ovf = 1;
            return;
        }
        const int id = cx.nV++;
        mirror_set(m, id, c);
        if (lane_id() == 0) {
            ws.gl[id] = c;
            ws.pa[id] = src;
            ws.td[id] = src;
        }
    } else if (src != 0 && !cx.reach_only) {
        if (cx.nX >= kSmallX) {
            cx.ovf = 1;
            return;
        }
        if (lane_id() == 0) ws.extra[cx.nX] = make_int2(src, l);
        ++cx.nX;
    }
}

// Claim every live edge the wave holds (per lane: `mask` over the targets in `col`, source
// `src`), one at a time, lowest lane and bit first.
__device__ __forceinline__ void claim_all(WaveState &ws, Mirror &m, SampleCtx &cx, uint32_t mask,
                                          uint4 col, int src)
{
    const int lane = lane_id();
    for (;;) {
        const unsigned long long pend = __ballot(mask != 0);
        if (!pend || cx.ovf) break;
        const int leader = (int)__builtin_ctzll(pend);
        const int myc = mask ? pick(col, __builtin_ctz(mask)) : 0;
        // direct reads of the leader's registers (no LDS round trip)
        const int c = __builtin_amdgcn_readlane(myc, leader);
        const int s = __builtin_amdgcn_readlane(src, leader);
        if (lane == leader) mask &= mask - 1;
        claim(ws, m, cx, c, s);
    }
}

// Seed level of sample j from the cache.
__device__ __forceinline__ void expand_seeds_cached(const SeedCache &sc, WaveState &ws, Mirror &m,
                                                    SampleCtx &cx, uint32_t j, uint32_t key_lo,
                                                    uint32_t key_hi)
{
    if (lane_id() == 0) cx.scanned += sc.scanned;
#pragma unroll
    for (int s = 0; s < kSeedSlots; ++s) {
        if (64 * s >= sc.total || cx.ovf) break;
        uint32_t mask = 0;
        if (sc.vmask[s]) {
            uint32_t w0, w1, w2, w3;
            philox4x32_10((uint32_t)sc.quad[s], j, key_lo, key_hi, w0, w1, w2, w3);
            const uint4 t = sc.thr[s];
            mask = ((w0 >> 8) < t.x ? 1u : 0u) | ((w1 >> 8) < t.y ? 2u : 0u) |
                   ((w2 >> 8) < t.z ? 4u : 0u) | ((w3 >> 8) < t.w ? 8u : 0u);
            mask &= sc.vmask[s];
        }
        cx.live += (uint32_t)__builtin_popcount(mask);
        claim_all(ws, m, cx, mask, sc.col[s], 0);
    }
}

// Expand frontier [lo, hi): seeds of the instance (source = merged seed 0) or local ids.
template <bool kLT>
__device__ void expand_small(const InstanceDesc &I, WaveState &ws, Mirror &m, SampleCtx &cx,
                             bool from_seeds, int lo, int hi, uint32_t j, uint32_t key_lo,
                             uint32_t key_hi, int quad_limit)
{
    const int lane = lane_id();
    for (int base = lo; base < hi && !cx.ovf; base += 64) {
        wave_sync();
        const int k = base + lane;
        int e0 = 0, e1 = 0;
        if (k < hi) {
            const int v = from_seeds ? I.seeds[k] : ws.gl[k];
            e0 = I.row_ptr[v];
            e1 = I.row_ptr[v + 1];
        }
        const int nq = quads_of(e0, e1);
        cx.scanned += (uint32_t)(e1 - e0);
        const int incl = wave_scan(nq);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        if (total > quad_limit) {  // a heavy frontier: the large kernel does this better
            cx.ovf = 1;
            return;
        }
        wave_sync();
        ws.e0[lane] = e0;
        ws.e1[lane] = e1;
        ws.ex[lane] = incl - nq;
        wave_sync();
        const int cnt = min(64, hi - base);
        for (int qb = 0; qb < total && !cx.ovf; qb += 64) {
            const int q = qb + lane;
            uint32_t mask = 0;
            uint4 col = make_uint4(0, 0, 0, 0);
            int src = 0;
            if (q < total) {
                int l = 0, h = cnt - 1;
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (ws.ex[mid] <= q) l = mid;
                    else h = mid - 1;
                }
                const int quad = (ws.e0[l] >> 2) + (q - ws.ex[l]);
                // both loads in flight at once: one memory round trip per level
                const uint4 thr = I.thr4[quad];
                col = I.col4[quad];
                if (kLT) {
                    const uint4 lo4 = I.lo4[quad];
                    mask = live_mask_lt(quad, j, key_lo, key_hi, ws.e0[l], ws.e1[l], lo4, thr, col);
                } else {
                    mask = live_mask(quad, j, key_lo, key_hi, ws.e0[l], ws.e1[l], thr);
                }
                src = from_seeds ? 0 : base + l;
            }
            cx.live += (uint32_t)__builtin_popcount(mask);
            claim_all(ws, m, cx, mask, col, src);
        }
    }
}

__device__ __forceinline__ int nca_small(const WaveState &ws, int x, int y, int &bad)
{
    while (x != y) {
        if (x > y) {
            const int nx = ws.td[x];
            if (nx < 0 || nx >= x) { bad = 1; return 0; }
            x = nx;
        } else {
            const int ny = ws.td[y];
            if (ny < 0 || ny >= y) { bad = 1; return 0; }
            y = ny;
        }
    }
    return x;
}

// One sample: BFS, dominators, subtree sizes into D. Returns false when it must be handed
// to the large kernel.
template <bool kLT>
__device__ bool run_sample(const SmallArgs &a, const InstanceDesc &I, const SeedCache &sc,
                           WaveState &ws, uint32_t j, Tally &tally)
{
    const int lane = lane_id();
    const unsigned long long key = (((unsigned long long)I.seed_hi << 32) | I.seed_lo) + a.round;
    const uint32_t key_lo = (uint32_t)key, key_hi = (uint32_t)(key >> 32);
    Mirror m;  // every row -1: nothing reached yet
    SampleCtx cx;
    cx.nV = 1;
    cx.nX = 0;
    cx.L = 1;
    cx.ovf = 0;
    cx.reach_only = a.reach_only;
    cx.live = 0;
    cx.scanned = 0;
    wave_sync();
    if (lane == 0) {
        ws.gl[0] = -1;
        ws.pa[0] = 0;
        ws.td[0] = 0;
        ws.lvl[0] = 0;
        ws.lvl[1] = 1;
    }
    wave_sync();
    if (!kLT && sc.total >= 0)
        expand_seeds_cached(sc, ws, m, cx, j, key_lo, key_hi);
    else
        expand_small<kLT>(I, ws, m, cx, true, 0, I.nseeds, j, key_lo, key_hi, a.quad_limit);
    int flo = 1, fhi = cx.nV;
    while (!cx.ovf && flo < fhi) {
        if (lane == 0) ws.lvl[cx.L + 1] = fhi;
        wave_sync();
        expand_small<kLT>(I, ws, m, cx, false, flo, fhi, j, key_lo, key_hi, a.quad_limit);
        flo = fhi;
        fhi = cx.nV;
        ++cx.L;
    }
    if (cx.ovf) return false;
    const int nV = cx.nV, nX = cx.nX, L = a.reach_only ? 1 : cx.L;
    wave_sync();

    // Dominator tree: Jacobi NCA steps over the extra edges (as in the workgroup kernel).
    int bad = 0;
    if (nX > 0) {
        for (int round = 0;; ++round) {
            for (int x = lane; x < nV; x += 64) ws.tn[x] = ws.td[x];
            wave_sync();
            for (int e = lane; e < nX; e += 64) {
                const int2 ed = ws.extra[e];
                const int tv = ws.td[ed.y];
                const int m1 = nca_small(ws, tv, ed.x, bad);
                const int m2 = nca_small(ws, tv, ws.pa[ed.y], bad);
                const int mm = min(m1, m2);
                if (mm < tv) atomicMin(&ws.tn[ed.y], mm);
            }
            wave_sync();
            int changed = 0;
            for (int x = lane; x < nV; x += 64) {
                const int nt = ws.tn[x];
                if (nt != ws.td[x]) {
                    ws.td[x] = nt;
                    changed = 1;
                }
            }
            wave_sync();
            if (!__any(changed) || __any(bad)) break;
            if (round >= kMaxSmallJacobiRounds) {
                bad = 1;
                break;
            }
        }
    }
    if (__any(bad)) {
        if (lane == 0) atomicOr(a.error, 2u);
        return true;  // never expected; reported through the error flag
    }

    // Subtree sizes, deepest BFS level first, accumulated into the instance's D.
    for (int x = lane; x < nV; x += 64) ws.tn[x] = 1;
    wave_sync();
    for (int l = L - 1; l >= 1; --l) {
        const int b0 = ws.lvl[l], b1 = ws.lvl[l + 1];
        for (int x = b0 + lane; x < b1; x += 64) {
            const int c = ws.tn[x];
            const int p = ws.td[x];
            if (p != 0) atomicAdd(&ws.tn[p], c);
            atomicAdd(&I.D[ws.gl[x]], (unsigned long long)c);
        }
        wave_sync();
    }
    tally.samples += 1;
    tally.reached += (unsigned long long)(nV - 1);
    tally.scanned += wave_sum(cx.scanned);
    tally.live += wave_sum(cx.live);
    return true;
}

template <bool kLT>
__global__ __launch_bounds__(kSmallBlock) void decrease_small_kernel(SmallArgs a)
{
    __shared__ SmallShared smem;
    const int lane = lane_id();
    WaveState &ws = smem.w[threadIdx.x >> 6];

    int cur = -1;
    InstanceDesc I{};
    uint32_t cur_lo = 0, cur_hi = 0;
    bool skip = false;  // the current instance's samples go straight to the large kernel
    bool done = false;  // many-instance launches: the instance's greedy run has ended
    SeedCache sc;
    sc.total = -1;
    Tally tally{0, 0, 0, 0};
    const uint32_t nwaves = gridDim.x * kSW;
    const uint32_t total = a.total;
    for (;;) {
        // Guided self-scheduling: runs of consecutive samples (one instance, one seed cache)
        // that shrink as the launch drains, so the waves finish together.
        uint32_t first = 0, want = kPickMin;
        if (lane == 0) {
            const uint32_t seen =
                __hip_atomic_load(a.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (seen < total)
                want = max(kPickMin,
                           min(kPickMax, (total - seen) / ((uint32_t)a.pick_div * nwaves)));
            first = atomicAdd(a.next, want);
        }
        first = __builtin_amdgcn_readfirstlane(__shfl(first, 0, 64));
        want = __builtin_amdgcn_readfirstlane(__shfl(want, 0, 64));
        if (first >= total) break;
        const uint32_t last = min(first + want, total);
        for (uint32_t idx = first; idx < last; ++idx) {
            int want_inst = cur;
            if (cur < 0 || idx < cur_lo || idx >= cur_hi) {
                // the last instance whose first sample index is <= idx
                int lo = 0, hi = a.ninst - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.inst[mid].sample_base <= idx) lo = mid;
                    else hi = mid - 1;
                }
                want_inst = __builtin_amdgcn_readfirstlane(lo);
            }
            if (want_inst != cur) {
                if (cur >= 0) flush(I, tally);
                cur = want_inst;
                I = a.inst[cur];
                cur_lo = I.sample_base;
                cur_hi = I.sample_base + I.theta;
                // Many-instance launches: an instance whose previous round handed most of
                // its samples over (control word set by the round's argmax) skips this
                // kernel; the results do not depend on which kernel runs a sample.
                skip = a.spill_inst &&
                       __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                           &I.ctrl[kCtrlSkipWave], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT)) != 0u;
                done = a.spill_inst &&
                       __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                           &I.ctrl[kCtrlDone], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT)) != 0u;
                if (done) skip = true;
                // LT: vertex-keyed choices, no quad cache
                if (kLT || skip) sc.total = -1;
                else build_seed_cache(I, ws.e0, ws.e1, ws.ex, sc);
            }
            const uint32_t j = idx - cur_lo;
            if (done) {
                // dropped: the rest of the run within this instance
                idx += min(last, cur_hi) - idx - 1;
                continue;
            }
            if (skip) {
                // the rest of the run within this instance, listed at once
                const uint32_t cnt = min(last, cur_hi) - idx;
                uint32_t pos = 0;
                if (lane == 0) pos = atomicAdd(a.spill_count, cnt);
                pos = __builtin_amdgcn_readfirstlane(__shfl(pos, 0, 64));
                for (uint32_t k = (uint32_t)lane; k < cnt; k += 64) {
                    a.spill_inst[pos + k] = (uint32_t)cur;
                    a.spill_j[pos + k] = j + k;
                }
                idx += cnt - 1;
                continue;
            }
            if (!run_sample<kLT>(a, I, sc, ws, j, tally) && lane == 0) {
                const uint32_t pos = atomicAdd(a.spill_count, 1u);
                if (a.spill_inst) {
                    a.spill_inst[pos] = (uint32_t)cur;
                    atomicAdd(&I.ctrl[kCtrlWaveHanded], 1u);  // this round's hand-overs
                }
                a.spill_j[pos] = j;
            }
        }
    }
    if (cur >= 0) flush(I, tally);
}

}  // namespace

hipError_t launch_decrease_small(const SmallArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipErrorInvalidValue;
    if (a.lt)
        hipLaunchKernelGGL(decrease_small_kernel<true>, dim3(grid), dim3(kSmallBlock), 0, stream, a);
    else
        hipLaunchKernelGGL(decrease_small_kernel<false>, dim3(grid), dim3(kSmallBlock), 0, stream,
                           a);
    return hipGetLastError();
}

}  // namespace imin
