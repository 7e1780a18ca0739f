// decrease.hip -- Algorithm 2 of arXiv 2302.13529 (DecreaseESComputation) on gfx950.
//
// One workgroup owns one scratch slot and takes samples j from a work counter until the
// launch's samples are exhausted. For sample j it:
//   1. decides live edges on the fly: edge e is live iff (W >> 8) < thr[e], W = word e&3 of
//      Philox4x32-10(counter (e>>2, j, 0, 0), key) -- nothing about the sample is stored
//      (Definition 4, live-edge sampling). One Philox call serves the 4 edges of a 32-byte
//      edge quad, and a lane works on one quad at a time;
//   2. runs a level-synchronous BFS from the merged seed (Section V, multiple seeds to one
//      seed) over live edges whose target is neither a seed nor blocked (Definition 2).
//      Reached vertices get local ids in BFS order; the BFS parent of each is kept, and
//      every other live edge between reached vertices is kept in an "extra" list;
//   3. computes the dominator tree of the reached subgraph (Section V-B3): starting from
//      the BFS tree t, it repeats the Jacobi step  t(v) <- NCA_t({t(v)} u pred(v))  for
//      every vertex with more than one reached predecessor until nothing changes. Each step
//      only moves t(v) up its current tree path, t(v) always precedes v in BFS order, the
//      tree always contains every dominator of v on the path of v, and a state where no
//      step changes anything is a solution of the dominator data-flow equations contained
//      in the true dominator sets, hence equal to them. The dominator tree is unique, so
//      this gives the same tree as Lengauer-Tarjan;
//   4. accumulates subtree sizes bottom-up over BFS levels (the immediate dominator of v is
//      on a strictly lower level) and adds each size to the exact 64-bit counter D[v]
//      (Algorithm 2's Delta[u] += c[u], Theorem 6, with the division by theta deferred).
//
// A sample whose scratch overflows is recorded and re-run by a second launch with
// large-capacity slots; its partial work is discarded, so results never depend on that.
#include "imin_internal.h"

namespace imin {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1,
                                              uint32_t &r0, uint32_t &r1, uint32_t &r2,
                                              uint32_t &r3)
{
    // Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3" (SC'11).
    // Counter words 2 and 3 are zero here.
    uint32_t x0 = c0, x1 = c1, x2 = 0u, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * x0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2);
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    r0 = x0;
    r1 = x1;
    r2 = x2;
    r3 = x3;
}

__device__ __forceinline__ bool bit_set(const uint32_t *bits, int v)
{
    return (bits[v >> 5] >> (v & 31)) & 1u;
}

// Exclusive prefix sum over the workgroup; *total receives the sum of all values.
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wave, int *total)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int s = s_wave[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    *total = tot;
    __syncthreads();
    return off + x - v;
}

struct SlotView {
    SlotEntry *map;
    int32_t *glob, *par0, *tdom, *tnew, *csz, *lvl;
    int2 *extra;
};

struct Shared {
    int src[kBlock];
    int e0[kBlock];
    int e1[kBlock];
    int qpre[kBlock + 1];
    int wave[kBlock / 64];
    unsigned idx;
    int tail;
    int nextra;
    int ovf;
    int changed;
};

__device__ __forceinline__ void visit(const DecreaseArgs &a, const SlotView &sv, Shared &sh,
                                      int w, int src, uint32_t epoch)
{
    const uint32_t old = __hip_atomic_exchange(&sv.map[w].stamp, epoch, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old != epoch) {
        const int id = atomicAdd(&sh.tail, 1);
        if (id < a.ws.lcap) {
            sv.map[w].lid = id;
            sv.glob[id] = w;
            sv.par0[id] = src;
            sv.tdom[id] = src;
            sv.csz[id] = 1;
        } else {
            sh.ovf = 1;
        }
    } else if (src != 0) {
        const int x = atomicAdd(&sh.nextra, 1);
        if (x < a.ws.xcap) sv.extra[x] = make_int2(src, w);
        else sh.ovf = 1;
    }
}

// Expand the frontier [lo, hi): seeds (from_seeds, source = merged root 0) or local ids.
__device__ void expand(const DecreaseArgs &a, const SlotView &sv, Shared &sh, bool from_seeds,
                       int lo, int hi, uint32_t j, uint32_t epoch, unsigned long long &scanned,
                       unsigned long long &live)
{
    const int tid = threadIdx.x;
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + tid;
        int nq = 0;
        if (k < hi) {
            const int v = from_seeds ? a.seeds[k] : sv.glob[k];
            const int src = from_seeds ? 0 : k;
            const int e0 = a.row_ptr[v];
            const int e1 = a.row_ptr[v + 1];
            scanned += (unsigned long long)(e1 - e0);
            nq = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
            sh.src[tid] = src;
            sh.e0[tid] = e0;
            sh.e1[tid] = e1;
        }
        int total;
        const int ex = block_exclusive_scan(nq, sh.wave, &total);
        sh.qpre[tid] = ex;
        __syncthreads();
        const int cnt = min(kBlock, hi - base);
        for (int q = tid; q < total; q += kBlock) {
            int l = 0, h = cnt - 1;
            while (l < h) {
                const int mid = (l + h + 1) >> 1;
                if (sh.qpre[mid] <= q) l = mid;
                else h = mid - 1;
            }
            const int e0 = sh.e0[l], e1 = sh.e1[l], src = sh.src[l];
            const int quad = (e0 >> 2) + (q - sh.qpre[l]);
            const uint4 p01 = a.edges[2 * (size_t)quad];
            const uint4 p23 = a.edges[2 * (size_t)quad + 1];
            uint32_t w0, w1, w2, w3;
            philox4x32_10((uint32_t)quad, j, a.key_lo, a.key_hi, w0, w1, w2, w3);
            const int eb = quad * 4;
            const uint32_t wv[4] = {w0, w1, w2, w3};
            const uint32_t cv[4] = {p01.x, p01.z, p23.x, p23.z};
            const uint32_t tv[4] = {p01.y, p01.w, p23.y, p23.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = eb + i;
                if (e < e0 || e >= e1) continue;
                if ((wv[i] >> 8) >= tv[i]) continue;
                const int c = (int)cv[i];
                if (bit_set(a.inelig, c)) continue;
                ++live;
                visit(a, sv, sh, c, src, epoch);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int nca(const int32_t *t, int x, int y)
{
    while (x != y) {
        if (x > y) x = t[x];
        else y = t[y];
    }
    return x;
}

__global__ __launch_bounds__(kBlock) void decrease_kernel(DecreaseArgs a)
{
    __shared__ Shared sh;
    const int tid = threadIdx.x;
    const size_t slot = blockIdx.x;
    SlotView sv;
    sv.map = a.ws.map + slot * (size_t)a.n;
    sv.glob = a.ws.glob + slot * (size_t)a.ws.lcap;
    sv.par0 = a.ws.par0 + slot * (size_t)a.ws.lcap;
    sv.tdom = a.ws.tdom + slot * (size_t)a.ws.lcap;
    sv.tnew = a.ws.tnew + slot * (size_t)a.ws.lcap;
    sv.csz = a.ws.csz + slot * (size_t)a.ws.lcap;
    sv.lvl = a.ws.lvl + slot * (size_t)(a.ws.lcap + 1);
    sv.extra = a.ws.extra + slot * (size_t)a.ws.xcap;
    uint32_t epoch = a.ws.epoch[slot];
    const uint32_t count = a.sample_list ? *a.sample_count : a.theta;

    unsigned long long t_samples = 0, t_reached = 0, t_scanned = 0, t_live = 0;

    for (;;) {
        if (tid == 0) sh.idx = atomicAdd(a.next, 1u);
        __syncthreads();
        const uint32_t idx = sh.idx;
        if (idx >= count) break;
        const uint32_t j = a.sample_list ? a.sample_list[idx] : idx;
        ++epoch;
        if (tid == 0) {
            sh.tail = 1;
            sh.nextra = 0;
            sh.ovf = 0;
            sv.lvl[0] = 0;
            sv.lvl[1] = 1;
            sv.glob[0] = -1;
            sv.par0[0] = 0;
            sv.tdom[0] = 0;
            sv.csz[0] = 0;
        }
        __syncthreads();

        unsigned long long p_scanned = 0, p_live = 0;
        expand(a, sv, sh, true, 0, a.nseeds, j, epoch, p_scanned, p_live);
        int L = 1, lo = 1;
        int hi = sh.tail;
        __syncthreads();
        while (lo < hi) {
            if (sh.ovf) break;
            if (tid == 0) sv.lvl[L + 1] = hi;
            expand(a, sv, sh, false, lo, hi, j, epoch, p_scanned, p_live);
            lo = hi;
            hi = sh.tail;
            ++L;
            __syncthreads();
        }
        if (sh.ovf) {
            if (tid == 0) {
                if (a.spill_ok) {
                    const uint32_t pos = atomicAdd(a.ovf_count, 1u);
                    a.ovf_list[pos] = j;
                    atomicAdd(&a.stats[4], 1ull);
                } else {
                    atomicOr(a.error, 1u);
                }
            }
            continue;
        }
        const int nV = sh.tail;
        const int nX = sh.nextra;

        // Extra edges: resolve the target vertex to its local id.
        for (int x = tid; x < nX; x += kBlock) {
            int2 e = sv.extra[x];
            e.y = sv.map[e.y].lid;
            sv.extra[x] = e;
        }
        __syncthreads();

        // Dominator tree: Jacobi NCA steps over vertices with several reached predecessors.
        if (nX > 0) {
            for (;;) {
                for (int x = tid; x < nX; x += kBlock) {
                    const int v = sv.extra[x].y;
                    sv.tnew[v] = sv.tdom[v];
                }
                if (tid == 0) sh.changed = 0;
                __syncthreads();
                for (int x = tid; x < nX; x += kBlock) {
                    const int2 e = sv.extra[x];
                    const int tv = sv.tdom[e.y];
                    const int m1 = nca(sv.tdom, tv, e.x);
                    const int m2 = nca(sv.tdom, tv, sv.par0[e.y]);
                    const int mm = min(m1, m2);
                    if (mm < tv)
                        __hip_atomic_fetch_min(&sv.tnew[e.y], mm, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                __syncthreads();
                for (int x = tid; x < nX; x += kBlock) {
                    const int v = sv.extra[x].y;
                    const int nv = sv.tnew[v];
                    if (nv != sv.tdom[v]) {
                        sv.tdom[v] = nv;
                        sh.changed = 1;
                    }
                }
                __syncthreads();
                const int ch = sh.changed;
                __syncthreads();
                if (!ch) break;
            }
        }

        // Subtree sizes, deepest BFS level first, and the exact accumulation into D.
        for (int l = L - 1; l >= 1; --l) {
            const int b0 = sv.lvl[l], b1 = sv.lvl[l + 1];
            for (int i = b0 + tid; i < b1; i += kBlock) {
                const int c = sv.csz[i];
                const int p = sv.tdom[i];
                if (p != 0)
                    __hip_atomic_fetch_add(&sv.csz[p], c, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                atomicAdd(&a.D[sv.glob[i]], (unsigned long long)c);
            }
            __syncthreads();
        }
        t_scanned += p_scanned;
        t_live += p_live;
        if (tid == 0) {
            t_samples += 1;
            t_reached += (unsigned long long)(nV - 1);
        }
    }
    if (tid == 0) a.ws.epoch[slot] = epoch;
    if (t_samples) atomicAdd(&a.stats[0], t_samples);
    if (t_reached) atomicAdd(&a.stats[1], t_reached);
    if (t_scanned) atomicAdd(&a.stats[2], t_scanned);
    if (t_live) atomicAdd(&a.stats[3], t_live);
}

}  // namespace

hipError_t launch_decrease(const DecreaseArgs &a, hipStream_t stream)
{
    if (a.ws.slots <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(decrease_kernel, dim3(a.ws.slots), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace imin
