// small.hip -- Algorithm 2 of arXiv 2302.13529 for samples that stay small: one wavefront per
// sample, every per-sample array in LDS, no block barrier anywhere.
//
// A wave takes a (instance, sample) pair from a work counter spanning all instances of the
// launch, so many graphs (the batched form) or one graph share the same launch. Per sample:
//   * live edges are decided per 4-edge quad with the same Philox4x32-10 coin as the large
//     kernel (Definition 4); lanes work on consecutive quads of the frontier;
//   * reachability from the merged seed is a wave-synchronous BFS. The live edges a wave
//     finds are claimed one at a time in lane order: the ids of the reached vertices are
//     mirrored in registers (4 per lane), so "already reached?" is one compare and a ballot;
//   * dominators use the same Jacobi NCA raising from the BFS tree as the large kernel, and
//     subtree sizes the same bottom-up pass over BFS levels (LDS atomics), with the sizes
//     added into the instance's 64-bit counters D (Algorithm 2, Theorem 6).
// A sample that reaches kSmallV - 1 vertices, keeps more than kSmallX extra edges, or meets a
// frontier with more than the launch's quad limit is abandoned (nothing accumulated) and
// listed for the large kernel, so results never depend on which path ran.
#include "imin_internal.h"
#include "philox.h"

namespace imin {
namespace {

constexpr int kSW = kSmallWaves;
constexpr int kSmallBlock = kSW * 64;
constexpr int kMaxSmallJacobiRounds = 4 * kSmallV;

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

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Orders this wave's LDS accesses across lanes (the hardware runs one wave's LDS
// instructions in order; this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Per-lane copy of the reached vertex ids: lane l holds local ids l, 64+l, 128+l, 192+l.
struct Mirror {
    int g[kSmallV / 64];
};

__device__ __forceinline__ void mirror_set(Mirror &m, int id, int v)
{
    if (lane_id() == (id & 63)) {
#pragma unroll
        for (int r = 0; r < kSmallV / 64; ++r)
            if ((id >> 6) == r) m.g[r] = v;
    }
}

// Local id of vertex c (uniform across the wave), or -1.
__device__ __forceinline__ int mirror_find(const Mirror &m, int c)
{
    int hit = -1;
#pragma unroll
    for (int r = 0; r < kSmallV / 64; ++r)
        if (m.g[r] == c) hit = r * 64 + lane_id();
    const unsigned long long b = __ballot(hit >= 0);
    if (!b) return -1;
    return __shfl(hit, (int)__builtin_ctzll(b), 64);
}

struct SampleCtx {
    int nV, nX, L;
    int ovf;
    uint32_t live, scanned;
};

// Claim live edge src -> c for the sample (c, src uniform across the wave).
__device__ __forceinline__ void claim(const InstanceDesc &I, WaveState &ws, Mirror &m,
                                      SampleCtx &cx, int c, int src)
{
    if ((I.inelig[c >> 5] >> (c & 31)) & 1u) return;  // seeds and blocked vertices
    ++cx.live;
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
    } else if (src != 0) {
        if (cx.nX >= kSmallX) {
            cx.ovf = 1;
            return;
        }
        if (lane_id() == 0) ws.extra[cx.nX] = make_int2(src, l);
        ++cx.nX;
    }
}

// Expand frontier [lo, hi): seeds of the instance (source = merged seed 0) or local ids.
__device__ void expand_small(const InstanceDesc &I, WaveState &ws, Mirror &m, SampleCtx &cx,
                             bool from_seeds, int lo, int hi, uint32_t j, uint32_t key_lo,
                             uint32_t key_hi, int quad_limit)
{
    const int lane = lane_id();
    for (int base = lo; base < hi && !cx.ovf; base += 64) {
        wave_sync();
        const int k = base + lane;
        int e0 = 0, e1 = 0, nq = 0;
        if (k < hi) {
            const int v = from_seeds ? I.seeds[k] : ws.gl[k];
            e0 = I.row_ptr[v];
            e1 = I.row_ptr[v + 1];
            nq = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
        }
        cx.scanned += (uint32_t)(e1 - e0);  // per-lane share, reduced by the caller
        int incl = nq;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, 63, 64);
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
                const uint4 thr = I.thr4[quad];
                mask = live_mask(quad, j, key_lo, key_hi, ws.e0[l], ws.e1[l], thr);
                if (mask) col = I.col4[quad];
                src = from_seeds ? 0 : base + l;
            }
            // claim the wave's live edges one at a time, lowest lane and bit first
            for (;;) {
                const unsigned long long pend = __ballot(mask != 0);
                if (!pend || cx.ovf) break;
                const int leader = (int)__builtin_ctzll(pend);
                int myc = 0;
                if (mask) {
                    const int i = __builtin_ctz(mask);
                    myc = (int)(i == 0 ? col.x : i == 1 ? col.y : i == 2 ? col.z : col.w);
                }
                const int c = __builtin_amdgcn_readfirstlane(__shfl(myc, leader, 64));
                const int s = __builtin_amdgcn_readfirstlane(__shfl(src, leader, 64));
                if (lane == leader) mask &= mask - 1;
                claim(I, ws, m, cx, c, s);
            }
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kSmallBlock) void decrease_small_kernel(SmallArgs a)
{
    __shared__ SmallShared smem;
    const int lane = lane_id();
    WaveState &ws = smem.w[threadIdx.x >> 6];

    for (;;) {
        uint32_t idx = 0;
        if (lane == 0) idx = atomicAdd(a.next, 1u);
        idx = __builtin_amdgcn_readfirstlane(__shfl(idx, 0, 64));
        if (idx >= a.total) break;
        // instance of this sample: the last one whose first sample index is <= idx
        int lo = 0, hi = a.ninst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.inst[mid].sample_base <= idx) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const InstanceDesc &I = a.inst[lo];
        const uint32_t j = idx - I.sample_base;
        const unsigned long long key =
            (((unsigned long long)I.seed_hi << 32) | I.seed_lo) + a.round;
        const uint32_t key_lo = (uint32_t)key, key_hi = (uint32_t)(key >> 32);

        Mirror m;
#pragma unroll
        for (int r = 0; r < kSmallV / 64; ++r) m.g[r] = -1;
        SampleCtx cx;
        cx.nV = 1;
        cx.nX = 0;
        cx.L = 1;
        cx.ovf = 0;
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
        expand_small(I, ws, m, cx, true, 0, I.nseeds, j, key_lo, key_hi, a.quad_limit);
        int flo = 1, fhi = cx.nV;
        while (!cx.ovf && flo < fhi) {
            if (lane == 0) ws.lvl[cx.L + 1] = fhi;
            wave_sync();
            expand_small(I, ws, m, cx, false, flo, fhi, j, key_lo, key_hi, a.quad_limit);
            flo = fhi;
            fhi = cx.nV;
            ++cx.L;
        }
        if (cx.ovf) {
            if (lane == 0) {
                const uint32_t pos = atomicAdd(a.spill_count, 1u);
                if (a.spill_inst) a.spill_inst[pos] = (uint32_t)lo;
                a.spill_j[pos] = j;
            }
            continue;
        }
        const int nV = cx.nV, nX = cx.nX, L = cx.L;
        wave_sync();

        // Dominator tree: Jacobi NCA steps over the extra edges (see decrease.hip).
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
            continue;
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
        const uint32_t scanned = wave_sum(cx.scanned);
        if (lane == 0) {
            atomicAdd(&I.stats[0], 1ull);
            atomicAdd(&I.stats[1], (unsigned long long)(nV - 1));
            atomicAdd(&I.stats[2], (unsigned long long)scanned);
            atomicAdd(&I.stats[3], (unsigned long long)cx.live);
            atomicAdd(&I.stats[5], 1ull);
        }
    }
}

}  // namespace

hipError_t launch_decrease_small(const SmallArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(decrease_small_kernel, dim3(grid), dim3(kSmallBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace imin
