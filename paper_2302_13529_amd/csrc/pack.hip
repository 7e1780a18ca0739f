// pack.hip -- Algorithm 2 of arXiv 2302.13529 for the smallest samples: kPackG samples of one
// instance share a wavefront, every per-sample array in LDS, no block barrier anywhere.
//
// Most samples of a sparse graph under small propagation probabilities reach a handful of
// vertices, so one sample leaves most lanes of a 64-lane wave idle. Here a wave runs a batch
// of kPackG consecutive samples of one instance side by side:
//   * the seed level comes from the register seed cache (every sample of an instance
//     expands the same seed rows; only the coins differ), each lane deciding its cached quads
//     for every sample of the batch (Definition 4, Philox4x32-10 per 4-edge quad); seed
//     rows beyond the cache are expanded from memory like a deeper level;
//   * deeper BFS levels form one flat work list over the frontiers of all samples of the
//     batch, and lanes take consecutive edge quads of it, each with its own sample's coins;
//   * a live edge is claimed in its sample's LDS hash table with one compare-and-swap: all
//     lanes claim at once, with no serial pass over the wave. The winner of a vertex gives it
//     the next local id of its sample (BFS parent = the edge's source); every other live edge
//     between reached vertices is kept as an extra edge, its target resolved to a local id
//     once the BFS is over. Local ids grow level by level, so the BFS tree and the level
//     boundaries are the same as in the other kernels;
//   * dominators use the same Jacobi NCA raising from the BFS tree (Section V-B3), and
//     subtree sizes the same bottom-up pass over BFS levels, over all samples of the batch
//     at once, with the sizes added into the instance's 64-bit counters D (Algorithm 2,
//     Theorem 6).
// A sample that reaches kPackV - 1 vertices, keeps more than kPackX extra edges, or expands a
// vertex with more edge quads than the quad limit is abandoned (nothing accumulated, its
// counters dropped) and listed for the workgroup kernel; results never depend on which
// kernel finished a sample.
#include "imin_internal.h"
#include "philox.h"
#include "wave.h"

namespace imin {
namespace {

using namespace wave;

constexpr int G = kPackG;
constexpr int V = kPackV;
constexpr int X = kPackX;
constexpr int H = kPackH;
constexpr int kHashBits = 7;
static_assert((1 << kHashBits) == H, "hash size");
static_assert(H >= 2 * V, "hash load");
constexpr int kPackBlock = kPackWaves * 64;
constexpr int kMaxJacobiRounds = 4 * V;
constexpr uint32_t kPickMin = 8;
constexpr uint32_t kPickMax = 64;

// LDS state of one sample of a batch. Local ids (< kPackV) and hash slots (< kPackH) fit a
// byte, which keeps a sample at about 1.6 KB so that LDS holds four waves per SIMD.
static_assert(V <= 256 && H <= 256, "byte-sized local ids and hash slots");
struct PackSample {
    int key[H];               // hash table of reached vertex ids (-1: empty)
    int gl[V];                // vertex id of each local id (local 0 is the merged seed: -1)
    int tn[V];                // next tentative dominator, then subtree sizes
    uint8_t hl[H];            // local id of the vertex in key[], written by the claim's winner
    uint8_t pa[V];            // parent in the BFS spanning tree
    uint8_t td[V];            // tentative immediate dominator
    uint8_t lvl[V + 4];       // first local id of each BFS level (V + 1 used)
    uint32_t extra[X];        // source local id | hash slot of the target << 8, then the
                              // target's local id << 8
    int nV, nX, ovf, pad;
};

struct PackWave {
    PackSample s[G];
    int e0[64], e1[64], ex[64], tag[64];  // flat frontier chunk: edge range, quad prefix,
                                          // (sample << 16) | local id
};

struct PackShared {
    PackWave w[kPackWaves];
};

__device__ __forceinline__ uint32_t hash_of(int c)
{
    return ((uint32_t)c * 2654435761u) >> (32 - kHashBits);
}

// Live edge src -> c of sample S (each lane its own edge and sample).
__device__ __forceinline__ void pclaim(PackSample &S, int c, int src)
{
    uint32_t h = hash_of(c);
    for (int p = 0; p < H; ++p) {
        const int old = atomicCAS(&S.key[h], -1, c);
        if (old == -1) {
            const int id = atomicAdd(&S.nV, 1);
            if (id < V) {
                S.gl[id] = c;
                S.pa[id] = (uint8_t)src;
                S.td[id] = (uint8_t)src;
                S.hl[h] = (uint8_t)id;
            } else {
                S.ovf = 1;
            }
            return;
        }
        if (old == c) {
            // edges from the merged seed never matter for dominators
            if (src != 0) {
                const int x = atomicAdd(&S.nX, 1);
                if (x < X) S.extra[x] = (uint32_t)src | (h << 8);
                else S.ovf = 1;
            }
            return;
        }
        h = (h + 1) & (H - 1);
    }
    S.ovf = 1;  // the table is full: more vertices than the sample may keep
}

__device__ __forceinline__ void claim_mask(PackSample &S, uint32_t mask, uint4 col, int src)
{
    while (mask) {
        const int i = __builtin_ctz(mask);
        mask &= mask - 1;
        pclaim(S, pick(col, i), src);
    }
}

// Per-lane counters of the G samples of a batch, indexed by a per-lane sample number
// without dynamic register indexing.
__device__ __forceinline__ void add_at(uint32_t (&a)[G], int g, uint32_t v)
{
#pragma unroll
    for (int t = 0; t < G; ++t) a[t] += (g == t) ? v : 0u;
}

// The sample and the offset of flat item k over per-sample ranges with prefix pre[].
__device__ __forceinline__ int flat_group(const int (&pre)[G + 1], int k)
{
    int g = 0;
#pragma unroll
    for (int t = 1; t < G; ++t) g += (k >= pre[t]) ? 1 : 0;
    return g;
}

__device__ __forceinline__ int pnca(const PackSample &S, int x, int y, int &bad)
{
    while (x != y) {
        if (x > y) {
            const int nx = S.td[x];
            if (nx < 0 || nx >= x) { bad = 1; return 0; }
            x = nx;
        } else {
            const int ny = S.td[y];
            if (ny < 0 || ny >= y) { bad = 1; return 0; }
            y = ny;
        }
    }
    return x;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One chunk of up to 64 frontier entries, one per lane: edge range [e0, e1) and tag
// (sample << 16) | source local id. Its edge quads are spread over the lanes, two in flight
// per lane, each with its own sample's coins, and the live edges are claimed.
__device__ __forceinline__ void expand_chunk(const InstanceDesc &I, PackWave &pw, int e0, int e1,
                                             int tag, int cnt, uint32_t j0, uint32_t key_lo,
                                             uint32_t key_hi, uint32_t (&live)[G])
{
    const int lane = lane_id();
    const int nq = quads_of(e0, e1);
    const int incl = wave_scan(nq);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    pw.e0[lane] = e0;
    pw.e1[lane] = e1;
    pw.ex[lane] = incl - nq;
    pw.tag[lane] = tag;
    wave_sync();
    // two quads per lane in flight: both loads issued before either is used
    for (int qb = 0; qb < total; qb += 128) {
        int g[2], src[2];
        uint32_t mask[2];
        uint4 col[2];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            const int q = qb + 64 * h2 + lane;
            mask[h2] = 0;
            col[h2] = make_uint4(0, 0, 0, 0);
            g[h2] = 0;
            src[h2] = 0;
            if (q < total) {
                int l = 0, h = cnt - 1;
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (pw.ex[mid] <= q) l = mid;
                    else h = mid - 1;
                }
                const int tg = pw.tag[l];
                g[h2] = tg >> 16;
                src[h2] = tg & 0xFFFF;
                if (pw.s[g[h2]].ovf == 0) {
                    const int quad = (pw.e0[l] >> 2) + (q - pw.ex[l]);
                    const uint4 thr = I.thr4[quad];
                    col[h2] = I.col4[quad];
                    mask[h2] = live_mask(quad, j0 + (uint32_t)g[h2], key_lo, key_hi, pw.e0[l],
                                         pw.e1[l], thr);
                }
            }
        }
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            add_at(live, g[h2], (uint32_t)__builtin_popcount(mask[h2]));
            claim_mask(pw.s[g[h2]], mask[h2], col[h2], src[h2]);
        }
    }
}

// Samples j0 .. j0 + k - 1 of instance I (k <= G). Returns the bit mask of the samples that
// finished; the others are to be handed over.
__device__ uint32_t run_batch(const PackArgs &a, const InstanceDesc &I, const SeedCache &sc,
                              PackWave &pw, uint32_t j0, int k, Tally &tally)
{
    const int lane = lane_id();
    const unsigned long long key = (((unsigned long long)I.seed_hi << 32) | I.seed_lo) + a.round;
    const uint32_t key_lo = (uint32_t)key, key_hi = (uint32_t)(key >> 32);

    wave_sync();
    for (int i = lane; i < G * H; i += 64) pw.s[i / H].key[i % H] = -1;
    if (lane < G) {
        PackSample &S = pw.s[lane];
        S.nV = 1;
        S.nX = 0;
        S.ovf = lane < k ? 0 : 2;
        S.gl[0] = -1;
        S.pa[0] = 0;
        S.td[0] = 0;
        S.lvl[0] = 0;
        S.lvl[1] = 1;
    }
    wave_sync();

    uint32_t live[G], scanned[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        live[g] = 0;
        scanned[g] = (lane == 0 && g < k) ? sc.scanned : 0u;
    }

    // Seed level, from the cache: every lane decides its cached quads for every sample.
#pragma unroll
    for (int s = 0; s < kSeedSlots; ++s) {
        if (64 * s >= sc.total) break;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g >= k) break;
            uint32_t mask = 0;
            if (sc.vmask[s]) {
                uint32_t w0, w1, w2, w3;
                philox4x32_10((uint32_t)sc.quad[s], j0 + (uint32_t)g, key_lo, key_hi, w0, w1,
                              w2, w3);
                const uint4 t = sc.thr[s];
                mask = ((w0 >> 8) < t.x ? 1u : 0u) | ((w1 >> 8) < t.y ? 2u : 0u) |
                       ((w2 >> 8) < t.z ? 4u : 0u) | ((w3 >> 8) < t.w ? 8u : 0u);
                mask &= sc.vmask[s];
            }
            live[g] += (uint32_t)__builtin_popcount(mask);
            claim_mask(pw.s[g], mask, sc.col[s], 0);
        }
    }
    wave_sync();

    // Seed level from memory when the seed rows do not fit the register cache: one flat
    // frontier of (sample, seed) entries whose source is the merged seed (local id 0). The
    // seeds' out-edges are already counted in sc.scanned, and no seed row is too heavy to
    // expand here (the rows are the same for every sample).
    if (sc.total < 0) {
        const int ns = I.nseeds;
        const int T = k * ns;
        for (int base = 0; base < T; base += 64) {
            wave_sync();
            const int kk = base + lane;
            int e0 = 0, e1 = 0, tag = 0;
            if (kk < T) {
                const int g = kk / ns;
                const int v = I.seeds[kk - g * ns];
                e0 = I.row_ptr[v];
                e1 = I.row_ptr[v + 1];
                tag = g << 16;
            }
            expand_chunk(I, pw, e0, e1, tag, min(64, T - base), j0, key_lo, key_hi, live);
        }
        wave_sync();
    }

    // Deeper levels: one flat frontier over the batch.
    int flo[G], fhi[G], L[G];
    bool act[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int nv = uni(pw.s[g].nV);
        const int ov = uni(pw.s[g].ovf);
        flo[g] = 1;
        fhi[g] = min(nv, V);
        L[g] = 1;
        act[g] = ov == 0 && nv <= V && flo[g] < fhi[g];
    }
    for (;;) {
        int pre[G + 1];
        pre[0] = 0;
        bool any = false;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (act[g] && lane == 0) pw.s[g].lvl[L[g] + 1] = (uint8_t)fhi[g];
            pre[g + 1] = pre[g] + (act[g] ? fhi[g] - flo[g] : 0);
            any = any || act[g];
        }
        if (!any) break;
        const int T = pre[G];
        for (int base = 0; base < T; base += 64) {
            wave_sync();
            const int kk = base + lane;
            int e0 = 0, e1 = 0, tag = 0;
            if (kk < T) {
                const int g = flat_group(pre, kk);
                int lid = kk - pre[0];
#pragma unroll
                for (int t = 0; t < G; ++t)
                    if (g == t) lid = flo[t] + (kk - pre[t]);
                const int v = pw.s[g].gl[lid];
                e0 = I.row_ptr[v];
                e1 = I.row_ptr[v + 1];
                tag = (g << 16) | lid;
                add_at(scanned, g, (uint32_t)(e1 - e0));
                if (quads_of(e0, e1) > a.quad_limit) {
                    pw.s[g].ovf = 1;  // a heavy vertex: the sample goes to a larger kernel
                    e1 = e0;
                }
            }
            expand_chunk(I, pw, e0, e1, tag, min(64, T - base), j0, key_lo, key_hi, live);
        }
        wave_sync();
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (!act[g]) continue;
            const int nv = uni(pw.s[g].nV);
            const int ov = uni(pw.s[g].ovf);
            if (ov != 0 || nv > V) {
                act[g] = false;
                continue;
            }
            flo[g] = fhi[g];
            fhi[g] = nv;
            ++L[g];
            act[g] = flo[g] < fhi[g];
        }
    }

    // The samples that finished their BFS within capacity.
    uint32_t okm = 0;
    int nV[G], nX[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        nV[g] = min(uni(pw.s[g].nV), V);
        nX[g] = min(uni(pw.s[g].nX), X);
        const bool ok = g < k && uni(pw.s[g].ovf) == 0 && uni(pw.s[g].nV) <= V &&
                        uni(pw.s[g].nX) <= X;
        if (ok) okm |= 1u << g;
        else nV[g] = nX[g] = 0;
    }

    // Extra edges: hash slot of the target -> its local id.
    int xpre[G + 1], vpre[G + 1];
    xpre[0] = vpre[0] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        xpre[g + 1] = xpre[g] + nX[g];
        vpre[g + 1] = vpre[g] + nV[g];
    }
    for (int kk = lane; kk < xpre[G]; kk += 64) {
        const int g = flat_group(xpre, kk);
        int x = kk;
#pragma unroll
        for (int t = 0; t < G; ++t)
            if (g == t) x = kk - xpre[t];
        PackSample &S = pw.s[g];
        const uint32_t e = S.extra[x];
        S.extra[x] = (e & 0xFFu) | ((uint32_t)S.hl[e >> 8] << 8);
    }
    wave_sync();

    // Dominator trees: Jacobi NCA steps over the extra edges of every sample at once.
    int bad = 0;
    if (xpre[G] > 0) {
        for (int round = 0;; ++round) {
            for (int kk = lane; kk < vpre[G]; kk += 64) {
                const int g = flat_group(vpre, kk);
                int v = kk;
#pragma unroll
                for (int t = 0; t < G; ++t)
                    if (g == t) v = kk - vpre[t];
                pw.s[g].tn[v] = pw.s[g].td[v];
            }
            wave_sync();
            for (int kk = lane; kk < xpre[G]; kk += 64) {
                const int g = flat_group(xpre, kk);
                int x = kk;
#pragma unroll
                for (int t = 0; t < G; ++t)
                    if (g == t) x = kk - xpre[t];
                PackSample &S = pw.s[g];
                const uint32_t e = S.extra[x];
                const int ex_src = (int)(e & 0xFFu), ex_dst = (int)(e >> 8);
                const int tv = S.td[ex_dst];
                const int m1 = pnca(S, tv, ex_src, bad);
                const int m2 = pnca(S, tv, S.pa[ex_dst], bad);
                const int mm = min(m1, m2);
                if (mm < tv) atomicMin(&S.tn[ex_dst], mm);
            }
            wave_sync();
            int changed = 0;
            for (int kk = lane; kk < vpre[G]; kk += 64) {
                const int g = flat_group(vpre, kk);
                int v = kk;
#pragma unroll
                for (int t = 0; t < G; ++t)
                    if (g == t) v = kk - vpre[t];
                PackSample &S = pw.s[g];
                const int nt = S.tn[v];
                if (nt != S.td[v]) {
                    S.td[v] = (uint8_t)nt;
                    changed = 1;
                }
            }
            wave_sync();
            if (!__any(changed) || __any(bad)) break;
            if (round >= kMaxJacobiRounds) {
                bad = 1;
                break;
            }
        }
    }
    if (__any(bad)) {
        if (lane == 0) atomicOr(a.error, 2u);
        return okm;  // never expected; reported through the error flag
    }

    // Subtree sizes, deepest BFS level first in every sample, accumulated into D.
    for (int kk = lane; kk < vpre[G]; kk += 64) {
        const int g = flat_group(vpre, kk);
        int v = kk;
#pragma unroll
        for (int t = 0; t < G; ++t)
            if (g == t) v = kk - vpre[t];
        pw.s[g].tn[v] = 1;
    }
    int maxL = 0;
#pragma unroll
    for (int g = 0; g < G; ++g)
        if ((okm >> g) & 1u) maxL = max(maxL, L[g]);
    wave_sync();
    for (int r = 0; r + 1 < maxL; ++r) {
        int lpre[G + 1], lbeg[G];
        lpre[0] = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int l = L[g] - 1 - r;
            int cnt = 0;
            lbeg[g] = 0;
            if (((okm >> g) & 1u) && l >= 1) {
                lbeg[g] = uni(pw.s[g].lvl[l]);
                cnt = uni(pw.s[g].lvl[l + 1]) - lbeg[g];
            }
            lpre[g + 1] = lpre[g] + cnt;
        }
        for (int kk = lane; kk < lpre[G]; kk += 64) {
            const int g = flat_group(lpre, kk);
            int v = kk;
#pragma unroll
            for (int t = 0; t < G; ++t)
                if (g == t) v = lbeg[t] + (kk - lpre[t]);
            PackSample &S = pw.s[g];
            const int c = S.tn[v];
            const int p = S.td[v];
            if (p != 0) atomicAdd(&S.tn[p], c);
            atomicAdd(&I.D[S.gl[v]], (unsigned long long)c);
        }
        wave_sync();
    }

#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t sc_g = wave_sum(scanned[g]);
        const uint32_t lv_g = wave_sum(live[g]);
        if ((okm >> g) & 1u) {
            tally.samples += 1;
            tally.reached += (unsigned long long)(nV[g] - 1);
            tally.scanned += sc_g;
            tally.live += lv_g;
        }
    }
    return okm;
}

__global__ __launch_bounds__(kPackBlock) void decrease_pack_kernel(PackArgs a)
{
    __shared__ PackShared smem;
    const int lane = lane_id();
    PackWave &pw = smem.w[threadIdx.x >> 6];

    int cur = -1;
    InstanceDesc I{};
    uint32_t cur_lo = 0, cur_hi = 0;
    bool skip = false;  // the current instance's samples go straight to the next kernel
    bool done = false;  // the current instance's greedy run has ended: its samples are dropped
    SeedCache sc;
    sc.total = -1;
    Tally tally{0, 0, 0, 0};
    // Guided self-scheduling of runs of consecutive samples (one instance, one seed cache)
    // that shrink as the launch drains. The remaining count is estimated from the counter
    // value the wave's previous claim returned, so a claim costs one device-scope atomic.
    const uint32_t nwaves = gridDim.x * kPackWaves;
    uint32_t seen = 0;
    for (;;) {
        uint32_t first = 0, last = 0;
        if (lane == 0) {
            const uint32_t want =
                seen < a.total
                    ? max(kPickMin, min(kPickMax, (a.total - seen) / ((uint32_t)a.pick_div * nwaves)))
                    : kPickMin;
            first = atomicAdd(a.next, want);
            seen = first + want;
            last = min(first + want, a.total);
        }
        first = __builtin_amdgcn_readfirstlane(__shfl(first, 0, 64));
        last = __builtin_amdgcn_readfirstlane(__shfl(last, 0, 64));
        if (first >= last) break;
        for (uint32_t idx = first; idx < last;) {
            if (cur < 0 || idx < cur_lo || idx >= cur_hi) {
                if (cur >= 0) flush(I, tally, true);
                int lo = 0, hi = a.ninst - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.inst[mid].sample_base <= idx) lo = mid;
                    else hi = mid - 1;
                }
                cur = __builtin_amdgcn_readfirstlane(lo);
                I = a.inst[cur];
                cur_lo = I.sample_base;
                cur_hi = I.sample_base + I.theta;
                // An instance whose samples mostly outgrew this kernel in an earlier round
                // skips it (control word set by the round's argmax). Seed rows that do not
                // fit the register cache are expanded from memory instead.
                skip = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                           &I.ctrl[kCtrlSkipPack], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT)) != 0u;
                done = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                           &I.ctrl[kCtrlDone], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT)) != 0u;
                if (done) {
                    sc.total = -1;
                } else if (!skip) {
                    build_seed_cache(I, pw.e0, pw.e1, pw.ex, sc);
                } else {
                    sc.total = -1;
                }
            }
            const uint32_t end = min(last, cur_hi);
            const uint32_t j0 = idx - cur_lo;
            if (done) {
                idx = end;
                continue;
            }
            if (skip) {
                const uint32_t cnt = end - idx;
                uint32_t pos = 0;
                if (lane == 0) pos = atomicAdd(a.out_count, cnt);
                pos = __builtin_amdgcn_readfirstlane(__shfl(pos, 0, 64));
                for (uint32_t q = (uint32_t)lane; q < cnt; q += 64) {
                    a.out_inst[pos + q] = (uint32_t)cur;
                    a.out_j[pos + q] = j0 + q;
                }
                idx = end;
                continue;
            }
            const int k = (int)min((uint32_t)G, end - idx);
            const uint32_t okm = run_batch(a, I, sc, pw, j0, k, tally);
            const uint32_t full = (1u << k) - 1u;
            if (okm != full && lane == 0) {
                const int nh = __builtin_popcount(full & ~okm);
                uint32_t pos = atomicAdd(a.out_count, (uint32_t)nh);
                for (int g = 0; g < k; ++g) {
                    if ((okm >> g) & 1u) continue;
                    a.out_inst[pos] = (uint32_t)cur;
                    a.out_j[pos] = j0 + (uint32_t)g;
                    ++pos;
                }
                atomicAdd(&I.ctrl[kCtrlPackHanded], (uint32_t)nh);
            }
            idx += (uint32_t)k;
        }
    }
    if (cur >= 0) flush(I, tally, true);
}

}  // namespace

hipError_t launch_decrease_pack(const PackArgs &a, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(decrease_pack_kernel, dim3(grid), dim3(kPackBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace imin
