// decrease.hip -- Algorithm 2 of arXiv 2302.13529 (DecreaseESComputation) on gfx950.
//
// One workgroup owns one scratch slot and takes samples j from a work counter until the
// launch's samples are exhausted. For sample j it:
//   1. decides live edges on the fly: edge e is live iff (W >> 8) < thr[e], W = word e&3 of
//      Philox4x32-10(counter (e>>2, j, 0, 0), key) -- nothing about the sample is stored
//      (Definition 4, live-edge sampling). One Philox call serves the 4 edges of a 32-byte
//      edge quad, and a lane works on one quad at a time. Under the linear-threshold model
//      (Section V-E) edge e = (v, u) is live iff u's choice falls in e's interval
//      [lo[e], thr[e]) (philox.h);
//   2. runs a level-synchronous BFS from the merged seed (Section V, multiple seeds to one
//      seed) over live edges. An edge into a seed or a blocked vertex (Definition 2) has
//      threshold 0 in the call's threshold array, so it is never live.
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
// A launch serves one problem, or many (batched calls, the query server): then every
// sample of its list names its instance, whose graph, thresholds, seeds, key and counters
// replace the launch's own.
#include "imin_internal.h"
#include "philox.h"

#include <algorithm>

namespace imin {
namespace {

// Exclusive prefix sum over a workgroup of B threads; *total receives the sum of all values.
template <int B>
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
    for (int w = 0; w < B / 64; ++w) {
        const int s = s_wave[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    *total = tot;
    __syncthreads();
    return off + x - v;
}

// The problem one sample belongs to.
struct Call {
    const int32_t *row_ptr;
    const uint4 *col4;
    const uint4 *edge;
    const uint4 *thr4;
    const uint4 *lo4;
    const uint4 *tl;
    const int32_t *seeds;
    int32_t nseeds;
    uint32_t key_lo, key_hi;
    unsigned long long *D;
    unsigned long long *stats;
};

struct SlotView {
    int2 *rng;  // row range of each local vertex (none in linear-threshold single calls)
    unsigned long long *map;
    LocalVtx *loc;
    int32_t *lvl;
    int2 *extra;
};

// Frontier entries per chunk: each of the B threads prepares kPerThread consecutive entries.
constexpr int kPerThread = 4;

template <int B>
struct Shared {
    static constexpr int kChunk = B * kPerThread;
    // local vertices whose dominator and subtree steps fit the frontier arrays' space
    static constexpr int kLdsV = kChunk + kChunk / 2;
    static_assert(kLdsV <= 65536, "16-bit local ids");
    union {
        struct {  // the BFS: one frontier chunk
            int e0[kChunk];
            int e1[kChunk];
            int qpre[kChunk + 1];
        };
        struct {  // afterwards, a sample of at most kLdsV local vertices
            int sz[kLdsV];         // subtree sizes (the Jacobi steps' next dominator meanwhile)
            uint16_t dom[kLdsV];   // tentative immediate dominators
            uint16_t par[kLdsV];   // BFS parents
        };
    };
    int wave[B / 64];
    unsigned idx;
    int tail;
    int nextra;
    int ovf;
    int changed;
    unsigned scanned;
    unsigned live;
};

// Live edge src -> w: w is claimed for this sample if it was not yet reached, or the edge is
// kept as an extra edge (edges from the merged seed never matter for dominators: their
// targets are its children). tag = this sample's epoch << lbits: every map entry written in
// this sample is at least tag, every older one below it.
// inc: 1 when the slot keeps reach counts in its map (the count word of w gains this
// sample's reach), else 0.
// kRng: w's row range r is kept with its local id, so that the next level starts from it
// without a dependent row_ptr read.
template <bool kRng, class Sh>
__device__ __forceinline__ void visit(const DecreaseArgs &a, const SlotView &sv, Sh &sh, int w,
                                      int src, uint32_t tag, uint32_t inc, int2 r)
{
    const unsigned long long tag64 = (unsigned long long)tag << 32;
    const unsigned long long old = __hip_atomic_fetch_max(&sv.map[w], tag64, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old < tag64) {
        const int id = atomicAdd(&sh.tail, 1);
        if (id < a.ws.lcap) {
            // a later max with tag64 leaves this larger value in place; the count word
            // (low) gains this sample's reach
            const uint32_t cnt = (uint32_t)old + inc;
            __hip_atomic_store(&sv.map[w],
                               ((unsigned long long)(tag | (uint32_t)(id + 1)) << 32) | cnt,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            LocalVtx rec;
            rec.glob = w;
            rec.par0 = src;
            rec.tdom = src;
            rec.csz = 1;
            sv.loc[id] = rec;
            if (kRng) sv.rng[id] = r;
        } else {
            // keep the slot's count (the sample is abandoned and re-run elsewhere)
            __hip_atomic_store(&sv.map[w], tag64 | (uint32_t)old, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
            sh.ovf = 1;
        }
    } else if (src != 0 && !a.reach_only) {
        const int x = atomicAdd(&sh.nextra, 1);
        if (x < a.ws.xcap) sv.extra[x] = make_int2(src, w);
        else sh.ovf = 1;
    }
}

// Quad q of the current chunk: the frontier entry it belongs to and its edge quad index.
template <class Sh>
__device__ __forceinline__ void locate(const Sh &sh, int cnt, int q, int &l, int &quad)
{
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.qpre[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    l = lo;
    quad = (sh.e0[lo] >> 2) + (q - sh.qpre[lo]);
}

// The live edges (mask) of one quad whose targets are in col. kRng: each target's row range
// is read from row_ptr beside its claim.
template <bool kRng, class Sh>
__device__ __forceinline__ void visit_mask(const DecreaseArgs &a, const SlotView &sv, Sh &sh,
                                           uint32_t mask, uint4 col, int src, uint32_t tag,
                                           uint32_t inc, uint32_t &live,
                                           const int32_t *row_ptr)
{
    live += (uint32_t)__builtin_popcount(mask);
    while (mask) {
        const int i = __builtin_ctz(mask);
        mask &= mask - 1;
        const uint32_t c = i == 0 ? col.x : i == 1 ? col.y : i == 2 ? col.z : col.w;
        int2 r = make_int2(0, 0);
        if (kRng) r = make_int2(row_ptr[c], row_ptr[c + 1]);
        visit<kRng>(a, sv, sh, (int)c, src, tag, inc, r);
    }
}

// The live edges (mask) of quad `quad` from their edge records (target, row start, row end):
// h holds the record of the lowest live edge; the next one is loaded while this one is
// claimed.
template <class Sh>
__device__ __forceinline__ void visit_edges(const DecreaseArgs &a, const SlotView &sv, Sh &sh,
                                            uint32_t mask, uint4 h, int quad, int src,
                                            uint32_t tag, uint32_t inc, uint32_t &live,
                                            const uint4 *edge)
{
    live += (uint32_t)__builtin_popcount(mask);
    while (mask) {
        mask &= mask - 1;
        const uint4 cur = h;
        if (mask) h = edge[((size_t)quad << 2) + __builtin_ctz(mask)];
        visit<true>(a, sv, sh, (int)cur.x, src, tag, inc, make_int2((int)cur.y, (int)cur.z));
    }
}

// Expand the frontier [lo, hi): seeds (from_seeds, source = merged root 0) or local ids.
// The frontier goes in chunks of B * kPerThread entries (kPerThread consecutive entries per
// thread);
// the edge quads of a chunk are spread evenly over the workgroup, two independent quads in
// flight per thread. A quad's thresholds are always read. Under IC only its live edges'
// records (target and row range) are read; under LT its targets are read first, since the
// coins depend on them, and a claimed target's row range comes from row_ptr in
// many-instance launches. kMulti: many-instance launch. Row ranges of local vertices are
// kept (kRng) except in linear-threshold single calls, which read row_ptr per frontier
// vertex.
template <int B, bool kLT, bool kMulti>
__device__ void expand(const DecreaseArgs &a, const Call &c, const SlotView &sv, Shared<B> &sh,
                       bool from_seeds, int lo, int hi, uint32_t j, uint32_t tag,
                       uint32_t inc, uint32_t &scanned, uint32_t &live)
{
    constexpr int kChunk = Shared<B>::kChunk;
    constexpr bool kRng = kMulti || !kLT;
    const int tid = threadIdx.x;
    for (int base = lo; base < hi; base += kChunk) {
        const int first = tid * kPerThread;
        int nq[kPerThread];
        int mine = 0;
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            const int k = base + first + i;
            nq[i] = 0;
            if (k < hi) {
                int e0, e1;
                if (kRng && !from_seeds) {
                    const int2 r = sv.rng[k];
                    e0 = r.x;
                    e1 = r.y;
                } else {
                    const int v = from_seeds ? c.seeds[k] : sv.loc[k].glob;
                    e0 = c.row_ptr[v];
                    e1 = c.row_ptr[v + 1];
                }
                scanned += (uint32_t)(e1 - e0);
                nq[i] = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
                sh.e0[first + i] = e0;
                sh.e1[first + i] = e1;
            }
            mine += nq[i];
        }
        int total;
        int ex = block_exclusive_scan<B>(mine, sh.wave, &total);
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            sh.qpre[first + i] = ex;
            ex += nq[i];
        }
        __syncthreads();
        const int cnt = min(kChunk, hi - base);
        for (int q = tid; q < total; q += 2 * B) {
            const int q2 = q + B;
            const bool has2 = q2 < total;
            int l1, quad1, l2, quad2;
            locate(sh, cnt, q, l1, quad1);
            locate(sh, cnt, has2 ? q2 : q, l2, quad2);
            const uint4 t1 = c.thr4[quad1];
            const uint4 t2 = c.thr4[quad2];
            if (kLT) {
                // a vertex-keyed choice per edge: the targets are needed first; they share
                // a 32-byte block with the quad's lower bounds
                const uint4 c1 = c.tl[2 * (size_t)quad1];
                const uint4 b1 = c.tl[2 * (size_t)quad1 + 1];
                const uint4 c2 = c.tl[2 * (size_t)quad2];
                const uint4 b2 = c.tl[2 * (size_t)quad2 + 1];
                const uint32_t m1 =
                    live_mask_lt(quad1, j, c.key_lo, c.key_hi, sh.e0[l1], sh.e1[l1], b1, t1, c1);
                const uint32_t m2 = has2 ? live_mask_lt(quad2, j, c.key_lo, c.key_hi, sh.e0[l2],
                                                        sh.e1[l2], b2, t2, c2)
                                         : 0u;
                visit_mask<kRng>(a, sv, sh, m1, c1, from_seeds ? 0 : base + l1, tag, inc, live,
                                 c.row_ptr);
                visit_mask<kRng>(a, sv, sh, m2, c2, from_seeds ? 0 : base + l2, tag, inc, live,
                                 c.row_ptr);
            } else {
                const uint32_t m1 =
                    live_mask(quad1, j, c.key_lo, c.key_hi, sh.e0[l1], sh.e1[l1], t1);
                const uint32_t m2 =
                    has2 ? live_mask(quad2, j, c.key_lo, c.key_hi, sh.e0[l2], sh.e1[l2], t2) : 0u;
                // the records of the lowest live edge of each quad, both in flight
                uint4 h1 = make_uint4(0, 0, 0, 0), h2 = make_uint4(0, 0, 0, 0);
                if (m1) h1 = c.edge[((size_t)quad1 << 2) + __builtin_ctz(m1)];
                if (m2) h2 = c.edge[((size_t)quad2 << 2) + __builtin_ctz(m2)];
                visit_edges(a, sv, sh, m1, h1, quad1, from_seeds ? 0 : base + l1, tag, inc, live,
                            c.edge);
                visit_edges(a, sv, sh, m2, h2, quad2, from_seeds ? 0 : base + l2, tag, inc, live,
                            c.edge);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int nca(const LocalVtx *t, int x, int y)
{
    while (x != y) {
        if (x > y) x = t[x].tdom;
        else y = t[y].tdom;
    }
    return x;
}

// The same walk over tentative dominators held in LDS.
__device__ __forceinline__ int nca_lds(const uint16_t *dom, int x, int y)
{
    while (x != y) {
        if (x > y) x = dom[x];
        else y = dom[y];
    }
    return x;
}

// Sum of a per-thread value over the wave, added into an LDS counter by lane 0.
__device__ __forceinline__ void wave_add(unsigned *dst, uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// B threads per workgroup: kBlock for single calls, kMultiBlock for many-instance launches,
// whose samples are mostly of moderate size and gain more from samples in flight.
template <bool kMulti, bool kLT, int B = kMulti ? kMultiBlock : kBlock>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(8, 8)))
void decrease_kernel(DecreaseArgs a)
{
    __shared__ Shared<B> sh;
    const int tid = threadIdx.x;
    const size_t slot = blockIdx.x;
    SlotView sv;
    sv.map = a.ws.map + slot * (size_t)a.ws.n;
    sv.loc = a.ws.loc + slot * (size_t)a.ws.lcap;
    sv.lvl = a.ws.lvl + slot * (size_t)(a.ws.lcap + 1);
    sv.extra = a.ws.extra + slot * (size_t)a.ws.xcap;
    sv.rng = (kMulti || !kLT) ? a.ws.rng + slot * (size_t)a.ws.lcap : nullptr;
    uint32_t epoch = a.ws.epoch[slot];
    const uint32_t emax = 0xFFFFFFFFu >> a.ws.lbits;  // largest epoch the map entries hold
    const uint32_t count = a.sample_list ? *a.sample_count : a.theta;
    // Reach counts in the map: every reached vertex's 1 rides on its claim, and
    // launch_flush_counts later adds the slot's whole map into D, n entries per slot. A slot
    // takes that route after its first sample when the samples it can expect to run
    // (count / slots of them, each about that size) reach at least n/4 vertices in all;
    // below that the flush would cost more than the D atomics it saves.
    const uint32_t per_slot = count / gridDim.x;
    bool cnt_on = false;

    for (;;) {
        if (tid == 0) sh.idx = atomicAdd(a.next, 1u);
        __syncthreads();
        const uint32_t idx = sh.idx;
        if (idx >= count) break;
        const uint32_t j = a.sample_list ? a.sample_list[idx] : idx;
        // This sample's problem: the launch's own, or an instance of a many-instance launch
        // (all instances' vertex ids fit the slot maps).
        Call c{a.row_ptr, a.col4,   a.edge,   a.thr4, a.lo4,  a.tl,
               a.seeds,   a.nseeds, a.key_lo, a.key_hi, a.D, a.stats};
        uint32_t inst_i = 0;
        if (kMulti) {
            inst_i = __builtin_amdgcn_readfirstlane(a.sample_inst[idx]);
            const InstanceDesc &I = a.inst[inst_i];
            const unsigned long long key =
                (((unsigned long long)I.seed_hi << 32) | I.seed_lo) + a.round;
            c = Call{I.row_ptr, I.col4,  I.edge,        I.thr4, I.lo4, I.tl, I.seeds,
                     I.nseeds, (uint32_t)key, (uint32_t)(key >> 32), I.D, I.stats};
        }
        if (epoch >= emax) {
            // every epoch value is used up: clear this slot's map (the barrier below orders
            // the stores before the sample's claims) and start again from epoch 1
            for (int64_t i = tid; i < a.ws.n; i += B)
                reinterpret_cast<uint32_t *>(&sv.map[i])[1] = 0u;
            epoch = 0;
        }
        ++epoch;
        const uint32_t tag = epoch << a.ws.lbits;
        if (tid == 0) {
            sh.tail = 1;
            sh.nextra = 0;
            sh.ovf = 0;
            sh.scanned = 0;
            sh.live = 0;
            sv.lvl[0] = 0;
            sv.lvl[1] = 1;
            LocalVtx root;
            root.glob = -1;
            root.par0 = 0;
            root.tdom = 0;
            root.csz = 0;
            sv.loc[0] = root;
        }
        __syncthreads();

        uint32_t p_scanned = 0, p_live = 0;
        const uint32_t inc = cnt_on ? 1u : 0u;
        expand<B, kLT, kMulti>(a, c, sv, sh, true, 0, c.nseeds, j, tag, inc, p_scanned, p_live);
        int L = 1, lo = 1;
        int hi = sh.tail;
        __syncthreads();
        while (lo < hi) {
            if (sh.ovf) break;
            if (tid == 0) sv.lvl[L + 1] = hi;
            expand<B, kLT, kMulti>(a, c, sv, sh, false, lo, hi, j, tag, inc, p_scanned, p_live);
            lo = hi;
            hi = sh.tail;
            ++L;
            __syncthreads();
        }
        if (sh.ovf) {
            // the sample is re-run elsewhere: take back the reach counts of its claims
            if (cnt_on) {
                const int nv = min(sh.tail, (int)a.ws.lcap);
                for (int i = 1 + tid; i < nv; i += B)
                    __hip_atomic_fetch_sub(reinterpret_cast<uint32_t *>(&sv.map[sv.loc[i].glob]),
                                           1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (tid == 0) {
                if (a.spill_ok) {
                    const uint32_t pos = atomicAdd(a.ovf_count, 1u);
                    a.ovf_list[pos] = j;
                    if (kMulti) a.ovf_inst[pos] = inst_i;
                    atomicAdd(&c.stats[4], 1ull);
                } else {
                    atomicOr(a.error, 1u);
                }
            }
            continue;
        }
        wave_add(&sh.scanned, p_scanned);
        wave_add(&sh.live, p_live);
        const int nV = sh.tail;
        const int nX = sh.nextra;
        if (a.reach_only) L = 1;  // reachability alone: no dominators, no counts

        // Extra edges: resolve the target vertex to its local id (an L2 read: the entry's
        // claim was an atomic there).
        const uint32_t lmask = (1u << a.ws.lbits) - 1u;
        for (int x = tid; x < nX; x += B) {
            int2 e = sv.extra[x];
            e.y = (int)((uint32_t)(__hip_atomic_load(&sv.map[e.y], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) >> 32) & lmask) - 1;
            sv.extra[x] = e;
        }
        __syncthreads();

        // A sample of at most kLdsV local vertices runs its dominator and subtree steps in
        // LDS: the frontier arrays' space is free once the BFS is done, and holds its
        // tentative dominators and BFS parents (16-bit local ids) and its subtree sizes. The
        // steps are those of the global form below; only where the three arrays live
        // differs.
        if (L > 1 && nV <= Shared<B>::kLdsV) {
            uint16_t *dom = sh.dom, *par = sh.par;
            int *sz = sh.sz;
            for (int i = tid; i < nV; i += B) {
                const LocalVtx r = sv.loc[i];
                dom[i] = (uint16_t)r.tdom;
                par[i] = (uint16_t)r.par0;
                sz[i] = 1;
            }
            __syncthreads();
            if (nX > 0) {
                for (int x0 = 0; x0 < nX; x0 += B) {
                    const int x = x0 + tid;
                    int2 e = make_int2(0, 0);
                    if (x < nX) {
                        e = sv.extra[x];
                        sz[e.y] = dom[e.y];
                    }
                    __syncthreads();
                    if (x < nX) {
                        const int tv = dom[e.y];
                        const int mm = min(nca_lds(dom, tv, e.x), nca_lds(dom, tv, par[e.y]));
                        if (mm < tv) atomicMin(&sz[e.y], mm);
                    }
                    __syncthreads();
                    if (x < nX) dom[e.y] = (uint16_t)sz[e.y];
                    __syncthreads();
                }
                for (;;) {
                    for (int x = tid; x < nX; x += B) {
                        const int v = sv.extra[x].y;
                        sz[v] = dom[v];
                    }
                    if (tid == 0) sh.changed = 0;
                    __syncthreads();
                    for (int x = tid; x < nX; x += B) {
                        const int2 e = sv.extra[x];
                        const int tv = dom[e.y];
                        const int mm = min(nca_lds(dom, tv, e.x), nca_lds(dom, tv, par[e.y]));
                        if (mm < tv) atomicMin(&sz[e.y], mm);
                    }
                    __syncthreads();
                    for (int x = tid; x < nX; x += B) {
                        const int v = sv.extra[x].y;
                        const int nv = sz[v];
                        if (nv != dom[v]) {
                            dom[v] = (uint16_t)nv;
                            sh.changed = 1;
                        }
                    }
                    __syncthreads();
                    const int ch = sh.changed;
                    __syncthreads();
                    if (!ch) break;
                }
                for (int x = tid; x < nX; x += B) sz[sv.extra[x].y] = 1;
                __syncthreads();
            }
            for (int l = L - 1; l >= 1; --l) {
                const int b0 = sv.lvl[l], b1 = sv.lvl[l + 1];
                for (int i = b0 + tid; i < b1; i += B) {
                    const int t = dom[i];
                    const int size = sz[i];
                    if (t != 0) atomicAdd(&sz[t], size);
                    const int add = cnt_on ? size - 1 : size;
                    if (add > 0) atomicAdd(&c.D[sv.loc[i].glob], (unsigned long long)add);
                }
                __syncthreads();
            }
        } else {
            // Dominator tree: Jacobi NCA steps over vertices with several reached predecessors.
            // The subtree-size field of such a vertex holds the next tentative dominator
            // meanwhile, and is reset to 1 afterwards.
            if (nX > 0) {
                // First one Gauss-Seidel sweep: the extra edges in list order (roughly the BFS
                // order of their sources), B at a time, each chunk one step over its targets on
                // the tree the earlier chunks left. A step over some vertices and some of their
                // predecessors keeps every dominator of v on v's tree path (a dominator of v
                // dominates each predecessor) and only moves t(v) up, so the Jacobi rounds below
                // still end at the dominator tree; they just have less left to change.
                for (int x0 = 0; x0 < nX; x0 += B) {
                    const int x = x0 + tid;
                    int2 e = make_int2(0, 0);
                    if (x < nX) {
                        e = sv.extra[x];
                        sv.loc[e.y].csz = sv.loc[e.y].tdom;
                    }
                    __syncthreads();
                    if (x < nX) {
                        const int tv = sv.loc[e.y].tdom;
                        const int m1 = nca(sv.loc, tv, e.x);
                        const int m2 = nca(sv.loc, tv, sv.loc[e.y].par0);
                        const int mm = min(m1, m2);
                        if (mm < tv)
                            __hip_atomic_fetch_min(&sv.loc[e.y].csz, mm, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    __syncthreads();
                    if (x < nX) sv.loc[e.y].tdom = sv.loc[e.y].csz;
                    __syncthreads();
                }
                for (;;) {
                    for (int x = tid; x < nX; x += B) {
                        const int v = sv.extra[x].y;
                        sv.loc[v].csz = sv.loc[v].tdom;
                    }
                    if (tid == 0) sh.changed = 0;
                    __syncthreads();
                    for (int x = tid; x < nX; x += B) {
                        const int2 e = sv.extra[x];
                        const int tv = sv.loc[e.y].tdom;
                        const int m1 = nca(sv.loc, tv, e.x);
                        const int m2 = nca(sv.loc, tv, sv.loc[e.y].par0);
                        const int mm = min(m1, m2);
                        if (mm < tv)
                            __hip_atomic_fetch_min(&sv.loc[e.y].csz, mm, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    __syncthreads();
                    for (int x = tid; x < nX; x += B) {
                        const int v = sv.extra[x].y;
                        const int nv = sv.loc[v].csz;
                        if (nv != sv.loc[v].tdom) {
                            sv.loc[v].tdom = nv;
                            sh.changed = 1;
                        }
                    }
                    __syncthreads();
                    const int ch = sh.changed;
                    __syncthreads();
                    if (!ch) break;
                }
                for (int x = tid; x < nX; x += B) sv.loc[sv.extra[x].y].csz = 1;
                __syncthreads();
            }

            // Subtree sizes, deepest BFS level first, and the exact accumulation into D.
            for (int l = L - 1; l >= 1; --l) {
                const int b0 = sv.lvl[l], b1 = sv.lvl[l + 1];
                for (int i = b0 + tid; i < b1; i += B) {
                    const LocalVtx r = sv.loc[i];
                    if (r.tdom != 0)
                        __hip_atomic_fetch_add(&sv.loc[r.tdom].csz, r.csz, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    // with reach counts in the map, a leaf of the dominator tree adds nothing here
                    const int add = cnt_on ? r.csz - 1 : r.csz;
                    if (add > 0) atomicAdd(&c.D[r.glob], (unsigned long long)add);
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            atomicAdd(&c.stats[0], 1ull);
            atomicAdd(&c.stats[1], (unsigned long long)(nV - 1));
            atomicAdd(&c.stats[2], (unsigned long long)sh.scanned);
            atomicAdd(&c.stats[3], (unsigned long long)sh.live);
        }
        if (a.count_reach && !cnt_on &&
            (unsigned long long)(nV - 1) * per_slot >= (unsigned long long)a.ws.n / 4)
            cnt_on = true;
    }
    if (tid == 0) {
        a.ws.epoch[slot] = epoch;
        if (a.count_reach) a.ws.dirty[slot] = cnt_on ? 1u : 0u;
    }
}

// D[v] += the reach counts of v in every slot that kept them (dirty), which go back to 0.
// Work items are (group of kFlushSlots slots, range of kFlushSpan vertices); a persistent
// grid walks them. Each workgroup first gathers the flags of all slots into LDS with one
// round of loads, so a launch in which no slot kept counts ends after that round. A thread
// owns one vertex of the range and has all its group's loads in flight at once; for each
// slot the threads of a wave read consecutive entries.
constexpr int kFlushSlots = 16;
constexpr int kFlushBlock = 256;
constexpr int kFlushSpan = 4 * kFlushBlock;
constexpr int kFlushGrid = 2048;
constexpr int kFlushMaxGroups = 256;  // slots <= 4096

__global__ __launch_bounds__(kFlushBlock) void flush_counts_kernel(
    unsigned long long *map, const uint32_t *dirty, int32_t slots, int64_t n,
    unsigned long long *D)
{
    __shared__ uint32_t gon[kFlushMaxGroups];
    __shared__ int any;
    const int32_t groups = (slots + kFlushSlots - 1) / kFlushSlots;
    for (int i = threadIdx.x; i < groups; i += kFlushBlock) gon[i] = 0;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < slots; s += kFlushBlock)
        if (dirty[s]) {
            atomicOr(&gon[s / kFlushSlots], 1u << (s % kFlushSlots));
            any = 1;
        }
    __syncthreads();
    if (!any) return;
    const int64_t spans = (n + kFlushSpan - 1) / kFlushSpan;
    for (int64_t item = blockIdx.x; item < spans * groups; item += gridDim.x) {
        const int32_t g = (int32_t)(item / spans);
        const uint32_t on = gon[g];
        if (!on) continue;
        const int32_t s0 = g * kFlushSlots;
        const int64_t v0 = (item - (int64_t)g * spans) * kFlushSpan;
        const int64_t v1 = min<int64_t>(v0 + kFlushSpan, n);
        for (int64_t v = v0 + threadIdx.x; v < v1; v += kFlushBlock) {
            uint32_t k[kFlushSlots];
#pragma unroll
            for (int i = 0; i < kFlushSlots; ++i)
                k[i] = (on >> i) & 1u
                           ? reinterpret_cast<const uint32_t *>(
                                 &map[(size_t)(s0 + i) * (size_t)n + (size_t)v])[0]
                           : 0u;
            unsigned long long sum = 0;
#pragma unroll
            for (int i = 0; i < kFlushSlots; ++i) {
                if (k[i]) {
                    sum += k[i];
                    reinterpret_cast<uint32_t *>(
                        &map[(size_t)(s0 + i) * (size_t)n + (size_t)v])[0] = 0u;
                }
            }
            if (sum) atomicAdd(&D[v], sum);
        }
    }
}

}  // namespace

hipError_t launch_flush_counts(const Workspace &ws, int32_t slots, unsigned long long *D,
                               hipStream_t stream)
{
    if (slots <= 0 || ws.n <= 0) return hipSuccess;
    if (slots > kFlushSlots * kFlushMaxGroups) return hipErrorInvalidValue;
    const int64_t items = ((ws.n + kFlushSpan - 1) / kFlushSpan) *
                          ((slots + kFlushSlots - 1) / kFlushSlots);
    const int grid = (int)std::min<int64_t>(kFlushGrid, items);
    hipLaunchKernelGGL(flush_counts_kernel, dim3(grid), dim3(kFlushBlock), 0, stream, ws.map,
                       ws.dirty, slots, ws.n, D);
    return hipGetLastError();
}

hipError_t launch_decrease(const DecreaseArgs &a, hipStream_t stream)
{
    if (a.ws.slots <= 0) return hipErrorInvalidValue;
    const dim3 grid(a.ws.slots);
    if (a.inst && a.lt)
        hipLaunchKernelGGL((decrease_kernel<true, true>), grid, dim3(kMultiBlock), 0, stream, a);
    else if (a.inst)
        hipLaunchKernelGGL((decrease_kernel<true, false>), grid, dim3(kMultiBlock), 0, stream, a);
    else if (a.lt)
        hipLaunchKernelGGL((decrease_kernel<false, true>), grid, dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((decrease_kernel<false, false>), grid, dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace imin
