// api.cpp -- host side of libimin: validation, device residency of the graph, scratch
// sizing, and the greedy drivers (Algorithms 3 and 4 of arXiv 2302.13529) as device-side
// round loops. Every step of the estimate runs in the kernels of decrease.hip/select.hip.
#include "graph.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using imin::DecreaseArgs;
using imin::Workspace;



namespace imin {
namespace host {

constexpr uint32_t kSpillSlots = 2;
constexpr int32_t kDefaultSmallWavesPerCu = 20;
constexpr int32_t kDefaultQuadLimit = 2048;
constexpr int32_t kDefaultPickDiv = 4;
// Packed kernel: a frontier vertex with more edge quads than this hands its sample over.
constexpr int32_t kDefaultPackQuadLimit = 256;
// Packed kernel workgroups per compute unit (kPackWaves waves of kPackG samples each): its
// registers allow 4 waves per SIMD, that is 4 workgroups.
constexpr int kPackGroupsPerCu = 4;

int pack_grid(int num_cus, const imin_launch &l)
{
    return std::max(1, num_cus) * (l.pack_per_cu > 0 ? l.pack_per_cu : kPackGroupsPerCu);
}
// In automatic mode the wave kernel is dropped for a graph once fewer than this share of
// a round's samples finished in it.
constexpr double kSmallKeepShare = 0.5;
// Workgroup-kernel slots while the wave kernel takes the samples first (it leaves few); a
// call whose first round leaves more than that grows them to the full count for the graph.
constexpr int32_t kSmallModeSlots = 64;


// ceil(p * 2^24) for p in [0, 1]; the product by a power of two is exact in fp32.
uint32_t live_threshold(float p)
{
    if (p <= 0.0f) return 0u;
    if (p >= 1.0f) return 1u << 24;
    return (uint32_t)std::ceil(p * 16777216.0f);
}


void free_ws(Workspace &ws)
{
    dfree(ws.map);
    dfree(ws.loc);
    dfree(ws.lvl);
    dfree(ws.extra);
    dfree(ws.rng);
    dfree(ws.epoch);
    dfree(ws.dirty);
    ws = Workspace();
}

size_t slot_bytes(int64_t n, int64_t lcap, int64_t xcap, bool rng = false)
{
    return (size_t)n * sizeof(unsigned long long) + (size_t)lcap * sizeof(imin::LocalVtx) +
           (size_t)(lcap + 1) * sizeof(int32_t) + (size_t)xcap * sizeof(int2) + 2 * sizeof(uint32_t) +
           (rng ? (size_t)lcap * sizeof(int2) : 0);
}

int alloc_ws(Workspace &ws, int64_t n, int32_t slots, int64_t lcap, int64_t xcap,
             hipStream_t stream, bool rng)
{
    if (ws.slots == slots && ws.n == n && ws.lcap == lcap && ws.xcap == xcap &&
        (ws.rng != nullptr) == rng)
        return IMIN_OK;
    free_ws(ws);
    // the map's local-id field holds lid + 1 <= lcap, and leaves at least one epoch bit
    int32_t lbits = 1;
    while (lbits < 32 && (int64_t(1) << lbits) <= lcap) ++lbits;
    if (lbits > 31) return IMIN_ERANGE;
    const size_t S = (size_t)slots;
    bool good = ok(hipMalloc(&ws.map, S * (size_t)n * sizeof(unsigned long long))) &&
                ok(hipMalloc(&ws.loc, S * (size_t)lcap * sizeof(imin::LocalVtx))) &&
                ok(hipMalloc(&ws.lvl, S * (size_t)(lcap + 1) * sizeof(int32_t))) &&
                ok(hipMalloc(&ws.extra, S * (size_t)std::max<int64_t>(xcap, 1) * sizeof(int2))) &&
                (!rng || ok(hipMalloc(&ws.rng, S * (size_t)lcap * sizeof(int2)))) &&
                ok(hipMalloc(&ws.epoch, S * sizeof(uint32_t))) &&
                ok(hipMalloc(&ws.dirty, S * sizeof(uint32_t)));
    if (!good) {
        free_ws(ws);
        (void)hipGetLastError();
        return IMIN_ENOMEM;
    }
    if (!ok(hipMemsetAsync(ws.map, 0, S * (size_t)n * sizeof(unsigned long long), stream)) ||
        !ok(hipMemsetAsync(ws.epoch, 0, S * sizeof(uint32_t), stream)) ||
        !ok(hipMemsetAsync(ws.dirty, 0, S * sizeof(uint32_t), stream))) {
        free_ws(ws);
        return IMIN_EDEVICE;
    }
    ws.slots = slots;
    ws.n = n;
    ws.lcap = lcap;
    ws.xcap = xcap;
    ws.lbits = lbits;
    ws.bytes = S * slot_bytes(n, lcap, xcap, rng);
    return IMIN_OK;
}

// Per-slot scratch: every local array holds all n vertices plus the root, so only the
// extra-edge list can overflow. Its default capacity covers a quarter of the vertices; a
// graph whose m is below that can never overflow and needs no spill path.
bool small_enabled(const imin_graph *g);

// max_slots > 0 caps a new allocation (an existing one of the right shape is kept).
int size_workspaces(imin_graph *g, int32_t max_slots)
{
    const int64_t lcap = (int64_t)g->n + 1;
    const int64_t xmax = (int64_t)g->m + 1;
    int64_t xcap = g->force_xcap > 0 ? g->force_xcap
                                     : std::max<int64_t>(4096, ((int64_t)g->n + 1) / 4);
    xcap = std::min(xcap, xmax);
    int32_t slots = g->force_slots;
    if (slots <= 0) {
        size_t free_b = 0, total_b = 0;
        if (!ok(hipMemGetInfo(&free_b, &total_b))) return IMIN_EDEVICE;
        free_b += g->main_ws.bytes;  // the current allocation is released before a new one
        const size_t per = slot_bytes(g->n, lcap, xcap, g->model == IMIN_IC);
        const size_t by_mem = std::max<size_t>(1, (free_b / 2) / per);
        slots = (int32_t)std::min<size_t>((size_t)imin::kSlotsPerCu * g->num_cus, by_mem);
        if (max_slots > 0) slots = std::min(slots, max_slots);
        // keep a working allocation that is at least as large, or a full-size one that the
        // free memory now sizes slightly differently
        const int32_t have = g->main_ws.slots;
        if (have > 0 && g->main_ws.lcap == lcap && g->main_ws.xcap == xcap &&
            (have >= slots || (max_slots == 0 && have > kSmallModeSlots)))
            slots = have;
    }
    // independent cascade: slots keep each claimed vertex's row range (from its edge record)
    const bool rng = g->model == IMIN_IC;
    int rc = alloc_ws(g->main_ws, g->n, slots, lcap, xcap, g->stream, rng);
    if (rc) return rc;
    if (xcap < xmax) {
        rc = alloc_ws(g->big_ws, g->n, kSpillSlots, lcap, xmax, g->stream, rng);
        if (rc) return rc;
    } else {
        free_ws(g->big_ws);
    }
    return IMIN_OK;
}

int prepare_workspaces(imin_graph *g)
{
    return size_workspaces(g, small_enabled(g) ? kSmallModeSlots : 0);
}

int ensure_ovf(imin_graph *g, uint32_t theta)
{
    if (theta <= g->ovf_cap) return IMIN_OK;
    dfree(g->d_ovf);
    if (!ok(hipMalloc(&g->d_ovf, (size_t)theta * sizeof(uint32_t)))) {
        g->ovf_cap = 0;
        return IMIN_ENOMEM;
    }
    g->ovf_cap = theta;
    return IMIN_OK;
}

int ensure_sj(imin_graph *g, uint32_t theta)
{
    if (theta <= g->sj_cap) return IMIN_OK;
    dfree(g->d_sj);
    if (!ok(hipMalloc(&g->d_sj, (size_t)theta * sizeof(uint32_t)))) {
        g->sj_cap = 0;
        return IMIN_ENOMEM;
    }
    g->sj_cap = theta;
    return IMIN_OK;
}

bool small_enabled(const imin_graph *g)
{
    if (g->small_mode == 0) return false;
    if (g->small_mode == 1) return true;
    return !g->small_auto_off;
}

int small_grid(int num_cus, const imin_launch &l)
{
    const int32_t wpc = l.waves_per_cu > 0 ? l.waves_per_cu : kDefaultSmallWavesPerCu;
    const int per_cu = std::max(1, (wpc + imin::kSmallWaves - 1) / imin::kSmallWaves);
    return num_cus * per_cu;
}

// The wave-kernel arguments that come from the launch shape.
void small_shape(imin::SmallArgs &s, const imin_launch &l)
{
    s.quad_limit = l.quad_limit > 0 ? l.quad_limit : kDefaultQuadLimit;
    s.pick_div = l.pick_div > 0 ? l.pick_div : kDefaultPickDiv;
}

bool launch_ok(const imin_launch *l)
{
    return !l || (l->waves_per_cu >= 0 && l->quad_limit >= 0 && l->pick_div >= 0 &&
                  (l->graph == 0 || l->graph == 1) && l->pack_per_cu >= -1);
}

int ensure_B(imin_graph *g, int32_t b)
{
    if (b <= g->B_cap) return IMIN_OK;
    dfree(g->d_B);
    if (!ok(hipMalloc(&g->d_B, (size_t)std::max(b, 1) * sizeof(int32_t)))) {
        g->B_cap = 0;
        return IMIN_ENOMEM;
    }
    g->B_cap = b;
    return IMIN_OK;
}

// Validated seed set: distinct seeds ascending, and the seed bitmap.
int seed_setup(imin_graph *g, const int32_t *S, int32_t nS, std::vector<int32_t> &seeds,
               std::vector<uint32_t> &inelig)
{
    if (!S || nS <= 0) return IMIN_EINVAL;
    inelig.assign((size_t)g->words, 0u);
    seeds.clear();
    for (int32_t i = 0; i < nS; ++i) {
        const int32_t s = S[i];
        if (s < 0 || s >= g->n) return IMIN_EINVAL;
        if (!((inelig[s >> 5] >> (s & 31)) & 1u)) {
            inelig[s >> 5] |= 1u << (s & 31);
            seeds.push_back(s);
        }
    }
    std::sort(seeds.begin(), seeds.end());
    return IMIN_OK;
}

// The graph as one instance of a wave-kernel launch (host copy in g->h_inst).
void describe(imin_graph *g, int32_t nseeds, uint64_t seed, uint32_t theta)
{
    imin::InstanceDesc &I = g->h_inst;
    I.row_ptr = g->d_row_ptr;
    I.col4 = g->d_col4;
    I.edge = g->d_edge;
    I.thr4 = g->d_thr4;
    I.lo4 = g->d_lo4;
    I.tl = g->d_tl;
    I.in_ptr = g->d_in_ptr;
    I.in_edge = g->d_in_edge;
    I.inelig = g->d_inelig;
    I.seeds = g->d_seeds;
    I.D = g->d_D;
    I.stats = g->d_stats;
    I.B = g->d_B;
    I.x = g->d_x;
    I.thr_orig = g->d_thr_orig;
    I.ctrl = g->d_ctrl;
    I.cand = g->d_cand;
    I.gr_k = -1;
    I.step = 0;
    I.nseeds = nseeds;
    I.n = g->n;
    I.nquads = (int32_t)std::max<int64_t>(((int64_t)g->m + 3) / 4, 1);
    I.seed_lo = (uint32_t)seed;
    I.seed_hi = (uint32_t)(seed >> 32);
    I.theta = theta;
    I.sample_base = 0;
}

// The vertices whose bit is set, ascending, appended to out (a word at a time).
void append_set_bits(const std::vector<uint32_t> &bits, std::vector<int32_t> &out)
{
    for (size_t w = 0; w < bits.size(); ++w) {
        uint32_t x = bits[w];
        while (x) {
            out.push_back((int32_t)(w * 32 + (size_t)__builtin_ctz(x)));
            x &= x - 1;
        }
    }
}

int upload_call_state(imin_graph *g, const std::vector<int32_t> &seeds,
                      const std::vector<uint32_t> &inelig, uint64_t seed, uint32_t theta)
{
    if (!ok(hipMemcpyAsync(g->d_seeds, seeds.data(), seeds.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, g->stream)) ||
        !ok(hipMemcpyAsync(g->d_inelig, inelig.data(), inelig.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, g->stream)))
        return IMIN_EDEVICE;
    if (!ok(imin::launch_fill_u64(g->d_stats, kStats, 0, g->stream)) ||
        !ok(imin::launch_fill_u32(g->d_ctrl, 4, 0, g->stream)))
        return IMIN_EDEVICE;
    describe(g, (int32_t)seeds.size(), seed, theta);
    if (!ok(hipMemcpyAsync(g->d_inst, &g->h_inst, sizeof(imin::InstanceDesc),
                           hipMemcpyHostToDevice, g->stream)))
        return IMIN_EDEVICE;
    // Working thresholds: restore the in-edges the previous call masked (all of them when
    // that call stopped half-way), then mask the in-edges of this call's seeds and blocked
    // vertices.
    uint32_t *thr = reinterpret_cast<uint32_t *>(g->d_thr4);
    const uint32_t *orig = reinterpret_cast<const uint32_t *>(g->d_thr_orig);
    g->mask_prev.swap(g->masked);
    if (!g->mask_known) {
        const int64_t quads = std::max<int64_t>(((int64_t)g->m + 3) / 4, 1);
        if (!ok(hipMemcpyAsync(g->d_thr4, g->d_thr_orig, (size_t)quads * sizeof(uint4),
                               hipMemcpyDeviceToDevice, g->stream)))
            return IMIN_EDEVICE;
    } else if (!g->mask_prev.empty()) {
        if (!ok(hipMemcpyAsync(g->d_list, g->mask_prev.data(),
                               g->mask_prev.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               g->stream)) ||
            !ok(imin::launch_mask_list(thr, orig, g->d_in_ptr, g->d_in_edge, g->d_list,
                                       (int32_t)g->mask_prev.size(), 1, g->stream)))
            return IMIN_EDEVICE;
    }
    g->mask_known = false;
    g->masked.clear();
    append_set_bits(inelig, g->masked);
    if (!g->masked.empty() &&
        (!ok(hipMemcpyAsync(g->d_list + g->n, g->masked.data(), g->masked.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, g->stream)) ||
         !ok(imin::launch_mask_list(thr, orig, g->d_in_ptr, g->d_in_edge, g->d_list + g->n,
                                    (int32_t)g->masked.size(), 0, g->stream))))
        return IMIN_EDEVICE;
    return IMIN_OK;
}

// The call ended with the seeds and `blockers` masked.
void end_masks(imin_graph *g, const std::vector<int32_t> &blockers)
{
    for (int32_t v : blockers) g->masked.push_back(v);
    g->mask_known = true;
}

uint32_t *thr_w(imin_graph *g) { return reinterpret_cast<uint32_t *>(g->d_thr4); }

// A fresh pair of timing events for one round's decrease launches.
int kernel_events(imin_graph *g, hipEvent_t *a, hipEvent_t *b)
{
    while (g->kev.size() < g->kev_used + 2) {
        hipEvent_t e;
        if (!ok(hipEventCreate(&e))) return IMIN_EDEVICE;
        g->kev.push_back(e);
    }
    *a = g->kev[g->kev_used];
    *b = g->kev[g->kev_used + 1];
    g->kev_used += 2;
    return IMIN_OK;
}

// The workgroup-per-sample kernel with Philox key `key` over samples 0..theta-1, or over
// the device list `list` of *count samples (at most theta), then the large-scratch launch
// for the samples that overflowed it. D and the stats accumulate: the main launch's slots
// decide one by one whether to keep reach counts in their maps (count_reach allows it),
// and the flush after the launches adds what they kept into D.
int launch_large_on(imin_graph *g, const LargeTarget &t, uint32_t theta, uint64_t key,
                    const uint32_t *list, const uint32_t *count, bool reach_only)
{
    const bool spill = t.big_ws->slots > 0;
    if (!ok(imin::launch_fill_u32(t.ctrl, 3, 0, g->stream))) return IMIN_EDEVICE;
    DecreaseArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->d_row_ptr;
    a.col4 = g->d_col4;
    a.edge = g->d_edge;
    a.thr4 = t.thr4;
    a.lo4 = g->d_lo4;
    a.tl = g->d_tl;
    a.lt = g->model == IMIN_LT ? 1 : 0;
    a.seeds = t.seeds;
    a.nseeds = t.nseeds;
    a.n = g->n;
    a.key_lo = (uint32_t)key;
    a.key_hi = (uint32_t)(key >> 32);
    a.theta = theta;
    a.sample_list = list;
    a.sample_count = count;
    a.next = t.ctrl + 0;
    a.D = t.D;
    a.stats = t.stats;
    a.ovf_list = t.ovf;
    a.ovf_count = t.ctrl + 2;
    a.error = t.ctrl + 3;
    a.spill_ok = spill ? 1 : 0;
    a.reach_only = reach_only ? 1 : 0;
    a.count_reach = reach_only ? 0 : 1;
    a.ws = *t.main_ws;
    a.ws.slots = (int32_t)std::min<uint32_t>((uint32_t)t.main_ws->slots, theta);
    const int32_t used = a.ws.slots;
    if (!ok(imin::launch_decrease(a, g->stream))) return IMIN_EDEVICE;
    if (spill) {
        a.sample_list = t.ovf;
        a.sample_count = t.ctrl + 2;
        a.next = t.ctrl + 1;
        a.spill_ok = 0;
        a.count_reach = 0;
        a.ws = *t.big_ws;
        if (!ok(imin::launch_decrease(a, g->stream))) return IMIN_EDEVICE;
    }
    if (!reach_only && !ok(imin::launch_flush_counts(*t.main_ws, used, t.D, g->stream)))
        return IMIN_EDEVICE;
    return IMIN_OK;
}

void multi_free(MultiScratch &ms)
{
    if (ms.exec) (void)hipGraphExecDestroy(ms.exec);
    ms.exec = nullptr;
    ms.exec_key.clear();
    dfree(ms.table);
    dfree(ms.stages);
    dfree(ms.stage);
    dfree(ms.rounds);
    dfree(ms.out);
    ms.table_cap = ms.stages_cap = ms.stage_cap = ms.rounds_cap = ms.out_cap = 0;
    free_ws(ms.main_ws);
    free_ws(ms.big_ws);
    dfree(ms.ctrl);
    dfree(ms.pi);
    dfree(ms.pj);
    dfree(ms.si);
    dfree(ms.sj);
    dfree(ms.oi);
    dfree(ms.oj);
    dfree(ms.part_d);
    dfree(ms.part_i);
    ms.n = ms.m = 0;
    ms.cap = 0;
    ms.inst_cap = 0;
}

int multi_alloc(MultiScratch &ms, int num_cus, int64_t max_n, int64_t max_m, uint32_t cap,
                int32_t max_inst, hipStream_t stream)
{
    const int64_t lcap = max_n + 1;
    const int64_t xmax = max_m + 1;
    const int64_t xcap = std::min<int64_t>(std::max<int64_t>(4096, lcap / 4), xmax);
    // kMultiSlotsPerCu workgroup slots per compute unit, within a quarter of the free memory
    size_t free_b = 0, total_b = 0;
    if (!ok(hipMemGetInfo(&free_b, &total_b))) return IMIN_EDEVICE;
    free_b += ms.main_ws.bytes;
    const size_t per = slot_bytes(max_n, lcap, xcap, true);
    const int32_t slots = (int32_t)std::max<size_t>(
        1, std::min<size_t>((size_t)imin::kMultiSlotsPerCu * std::max(1, num_cus),
                            (free_b / 4) / per));
    int rc = alloc_ws(ms.main_ws, max_n, slots, lcap, xcap, stream, true);
    if (rc) return rc;
    if (xcap < xmax) {
        rc = alloc_ws(ms.big_ws, max_n, (int32_t)kSpillSlots, lcap, xmax, stream, true);
        if (rc) return rc;
    } else {
        free_ws(ms.big_ws);
    }
    if (cap > ms.cap) {
        dfree(ms.pi);
        dfree(ms.pj);
        dfree(ms.si);
        dfree(ms.sj);
        dfree(ms.oi);
        dfree(ms.oj);
        ms.cap = 0;
        if (!ok(hipMalloc(&ms.pi, (size_t)cap * sizeof(uint32_t))) ||
            !ok(hipMalloc(&ms.pj, (size_t)cap * sizeof(uint32_t))) ||
            !ok(hipMalloc(&ms.si, (size_t)cap * sizeof(uint32_t))) ||
            !ok(hipMalloc(&ms.sj, (size_t)cap * sizeof(uint32_t))) ||
            !ok(hipMalloc(&ms.oi, (size_t)cap * sizeof(uint32_t))) ||
            !ok(hipMalloc(&ms.oj, (size_t)cap * sizeof(uint32_t)))) {
            (void)hipGetLastError();
            return IMIN_ENOMEM;
        }
        ms.cap = cap;
    }
    if (max_inst > ms.inst_cap) {
        dfree(ms.part_d);
        dfree(ms.part_i);
        ms.inst_cap = 0;
        const size_t parts = (size_t)max_inst * imin::kArgParts;
        if (!ok(hipMalloc(&ms.part_d, parts * sizeof(unsigned long long))) ||
            !ok(hipMalloc(&ms.part_i, parts * sizeof(int32_t)))) {
            (void)hipGetLastError();
            return IMIN_ENOMEM;
        }
        ms.inst_cap = max_inst;
    }
    if (!ms.ctrl && !ok(hipMalloc(&ms.ctrl, kMultiCtrl * sizeof(uint32_t)))) {
        (void)hipGetLastError();
        return IMIN_ENOMEM;
    }
    if (!ok(imin::launch_fill_u32(ms.ctrl, kMultiCtrl, 0, stream))) return IMIN_EDEVICE;
    ms.n = max_n;
    ms.m = max_m;
    return IMIN_OK;
}

int32_t gr_candidates(const imin_graph *g, const std::vector<int32_t> &seeds,
                      const std::vector<uint32_t> &inelig, std::vector<uint32_t> &cand)
{
    cand.assign((size_t)g->words, 0u);
    int32_t ncb = 0;
    for (int32_t s : seeds) {
        for (int32_t e = g->row_ptr[s]; e < g->row_ptr[s + 1]; ++e) {
            const int32_t v = g->col[e];
            const bool is_seed = (inelig[v >> 5] >> (v & 31)) & 1u;
            if (!is_seed && !((cand[v >> 5] >> (v & 31)) & 1u)) {
                cand[v >> 5] |= 1u << (v & 31);
                ++ncb;
            }
        }
    }
    return ncb;
}

int multi_round(MultiScratch &ms, const imin::InstanceDesc *inst, int32_t ninst, uint32_t total,
                uint32_t round, const imin_launch &shape, int num_cus, bool select, bool gr,
                bool lt, hipStream_t stream)
{
    if (total > ms.cap) return IMIN_ERANGE;
    const bool spill = ms.big_ws.slots > 0;
    // words 0-5, 7 and 8 restart every round; the error words 2 and 6 accumulate, and word 9
    // (instances done) over the call
    if (!ok(imin::launch_batch_zero(inst, ninst, stream)) ||
        !ok(imin::launch_fill_u32(ms.ctrl, 2, 0, stream)) ||
        !ok(imin::launch_fill_u32(ms.ctrl + 3, 3, 0, stream)) ||
        !ok(imin::launch_fill_u32(ms.ctrl + 7, 2, 0, stream)))
        return IMIN_EDEVICE;
    if (gr && !ok(imin::launch_batch_gr_prepare(inst, ninst, (int32_t)round, stream)))
        return IMIN_EDEVICE;
    // The smallest samples first, several to a wavefront (independent cascade only: the
    // packed kernel keeps the seed level's edge coins in registers); what outgrows it goes
    // straight to the workgroup kernel through a device-side list. The hand-overs are the
    // few larger samples (over 63 vertices or 64 extra edges), which the workgroup kernel's
    // 2048 slots finish sooner than one wavefront each would. Without the packed kernel
    // (linear threshold, or switched off) the one-sample-per-wave kernel takes every sample
    // first and hands its overflow on.
    const bool pack = !lt && shape.pack_per_cu >= 0;
    if (pack) {
        imin::PackArgs p;
        std::memset(&p, 0, sizeof(p));
        p.inst = inst;
        p.ninst = ninst;
        p.total = total;
        p.round = round;
        p.quad_limit = kDefaultPackQuadLimit;
        p.pick_div = shape.pick_div > 0 ? shape.pick_div : kDefaultPickDiv;
        p.next = ms.ctrl + 8;
        p.out_inst = ms.pi;
        p.out_j = ms.pj;
        p.out_count = ms.ctrl + 7;
        p.error = ms.ctrl + 2;
        if (!ok(imin::launch_decrease_pack(p, pack_grid(num_cus, shape), stream))) return IMIN_EDEVICE;
    }
    imin::SmallArgs s;
    std::memset(&s, 0, sizeof(s));
    s.inst = inst;
    s.ninst = ninst;
    s.total = total;
    s.round = round;
    small_shape(s, shape);
    s.lt = lt ? 1 : 0;
    s.next = ms.ctrl + 0;
    s.spill_inst = ms.si;
    s.spill_j = ms.sj;
    s.spill_count = ms.ctrl + 1;
    s.error = ms.ctrl + 2;
    if (!pack && !ok(imin::launch_decrease_small(s, small_grid(num_cus, shape), stream)))
        return IMIN_EDEVICE;
    DecreaseArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = (int32_t)ms.n;
    a.theta = total;
    a.sample_list = pack ? ms.pj : ms.sj;
    a.sample_count = pack ? ms.ctrl + 7 : ms.ctrl + 1;
    a.next = ms.ctrl + 3;
    a.ovf_list = ms.oj;
    a.ovf_count = ms.ctrl + 5;
    a.error = ms.ctrl + 6;
    a.spill_ok = spill ? 1 : 0;
    a.ws = ms.main_ws;
    a.inst = inst;
    a.sample_inst = pack ? ms.pi : ms.si;
    a.ovf_inst = ms.oi;
    a.round = round;
    a.lt = lt ? 1 : 0;
    if (!ok(imin::launch_decrease(a, stream))) return IMIN_EDEVICE;
    if (spill) {
        a.sample_list = ms.oj;
        a.sample_inst = ms.oi;
        a.sample_count = ms.ctrl + 5;
        a.next = ms.ctrl + 4;
        a.spill_ok = 0;
        a.ws = ms.big_ws;
        if (!ok(imin::launch_decrease(a, stream))) return IMIN_EDEVICE;
    }
    if (select) {
        if (ninst > ms.inst_cap) return IMIN_ERANGE;
        if (!ok(imin::launch_batch_argmax(inst, ninst, (int32_t)round, ms.part_d, ms.part_i,
                                          ms.ctrl + 9, stream)))
            return IMIN_EDEVICE;
    }
    return IMIN_OK;
}

int multi_errors(MultiScratch &ms, uint32_t *wave_err, uint32_t *wg_err, hipStream_t stream)
{
    uint32_t w[7];
    if (!ok(hipMemcpyAsync(w, ms.ctrl, sizeof(w), hipMemcpyDeviceToHost, stream)) ||
        !ok(hipStreamSynchronize(stream)))
        return IMIN_EDEVICE;
    *wave_err = w[2];
    *wg_err = w[6];
    return IMIN_OK;
}

// The graph's own call state as the target of the workgroup kernel.
int launch_large(imin_graph *g, int32_t nseeds, uint32_t theta, uint64_t key,
                 const uint32_t *list, const uint32_t *count, bool reach_only = false)
{
    LargeTarget t{g->d_thr4, g->d_seeds, nseeds, g->d_D, g->d_stats, g->d_ctrl, g->d_ovf,
                  &g->main_ws, &g->big_ws};
    return launch_large_on(g, t, theta, key, list, count, reach_only);
}

// One call of Algorithm 2 with Philox key seed + call, leaving D on the device. With the
// wave kernel on, it runs every sample first and leaves the ones that outgrow it to the
// workgroup kernel, through a device-side list (no host round trip).
int decrease_round(imin_graph *g, int32_t nseeds, uint32_t theta, uint64_t seed, uint32_t call,
                   bool reach_only = false)
{
    int rc = IMIN_OK;
    if (g->probe == 2) {
        // Automatic mode, a call that kept the wave kernel: after a timed round with it, a
        // timed trial round of the workgroup kernel alone, at its full slot count.
        g->small_auto_off = true;
        rc = size_workspaces(g, 0);
        if (rc) return rc;
    } else if (g->probe == 3) {
        // The call keeps whichever form ran its round faster (results are the same).
        g->probe = 0;
        const size_t a = g->probe_kev[0], b = g->probe_kev[1];
        float with = 0.0f, without = 0.0f;
        if (!ok(hipEventSynchronize(g->kev[b + 1])) ||
            !ok(hipEventElapsedTime(&with, g->kev[a], g->kev[a + 1])) ||
            !ok(hipEventElapsedTime(&without, g->kev[b], g->kev[b + 1])))
            return IMIN_EDEVICE;
        g->small_auto_off = without < with;
    }
    const bool small = small_enabled(g);
    if ((!reach_only && !ok(imin::launch_fill_u64(g->d_D, g->n, 0, g->stream))) ||
        (small && !ok(imin::launch_fill_u32(g->d_sctrl, 2, 0, g->stream))))
        return IMIN_EDEVICE;
    hipEvent_t k0, k1;
    rc = kernel_events(g, &k0, &k1);
    if (rc) return rc;
    if (g->probe == 1 || g->probe == 2) {
        g->probe_kev[g->probe - 1] = g->kev_used - 2;
        ++g->probe;
    }
    if (!ok(hipEventRecord(k0, g->stream))) return IMIN_EDEVICE;
    if (small) {
        imin::SmallArgs s;
        std::memset(&s, 0, sizeof(s));
        s.inst = g->d_inst;
        s.ninst = 1;
        s.total = theta;
        s.round = call;
        small_shape(s, g->small_launch);
        s.reach_only = reach_only ? 1 : 0;
        s.lt = g->model == IMIN_LT ? 1 : 0;
        s.next = g->d_sctrl + 0;
        s.spill_inst = nullptr;
        s.spill_j = g->d_sj;
        s.spill_count = g->d_sctrl + 1;
        s.error = g->d_ctrl + 3;
        if (!ok(imin::launch_decrease_small(s, small_grid(g->num_cus, g->small_launch),
                                            g->stream)))
            return IMIN_EDEVICE;
        if (g->auto_pending) {
            // First round of the call. When the wave kernel handed over more samples than
            // the workgroup kernel has slots, that kernel gets its full slot count now (the
            // samples it receives are the large ones). In automatic mode, when it handed
            // over most samples, the wave kernel also sits out the call's later rounds.
            // Results are the same either way.
            g->auto_pending = false;
            uint32_t handed = 0;
            if (!ok(hipMemcpyAsync(&handed, g->d_sctrl + 1, sizeof(handed),
                                   hipMemcpyDeviceToHost, g->stream)) ||
                !ok(hipStreamSynchronize(g->stream)))
                return IMIN_EDEVICE;
            const bool drop = g->small_mode == -1 &&
                              (double)handed > (1.0 - kSmallKeepShare) * (double)theta;
            if (drop) g->small_auto_off = true;
            if (g->small_mode == -1 && !drop && !reach_only) {
                // kept: the next round is timed with the wave kernel (this one waited for
                // the host), the one after it without
                g->probe = 1;
            }
            if (drop || handed > (uint32_t)g->main_ws.slots) {
                rc = size_workspaces(g, 0);
                if (rc) return rc;
            }
        }
        rc = launch_large(g, nseeds, theta, seed + call, g->d_sj, g->d_sctrl + 1, reach_only);
    } else {
        rc = launch_large(g, nseeds, theta, seed + call, nullptr, nullptr, reach_only);
    }
    if (rc) return rc;
    if (!ok(hipEventRecord(k1, g->stream))) return IMIN_EDEVICE;
    return IMIN_OK;
}

// Copies the stats and the error flag back; returns IMIN_EDEVICE if a sample was lost.
int finish_call(imin_graph *g, imin_stats *stats)
{
    unsigned long long st[kStats];
    uint32_t ctrl[4];
    if (!ok(hipMemcpyAsync(st, g->d_stats, sizeof(st), hipMemcpyDeviceToHost, g->stream)) ||
        !ok(hipMemcpyAsync(ctrl, g->d_ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, g->stream)) ||
        !ok(hipEventRecord(g->ev1, g->stream)) || !ok(hipEventSynchronize(g->ev1)))
        return IMIN_EDEVICE;
    if (ctrl[3] != 0) return IMIN_EDEVICE;
    if (stats) {
        float ms = 0.0f;
        if (!ok(hipEventElapsedTime(&ms, g->ev0, g->ev1))) return IMIN_EDEVICE;
        stats->samples = st[0];
        stats->reached = st[1];
        stats->edges_scanned = st[2];
        stats->live_edges = st[3];
        stats->spilled = st[4];
        stats->wave_samples = st[5];
        stats->pack_samples = st[6];
        stats->device_ms = ms;
        double kms = 0.0;
        for (size_t i = 0; i + 1 < g->kev_used; i += 2) {
            float x = 0.0f;
            if (!ok(hipEventElapsedTime(&x, g->kev[i], g->kev[i + 1]))) return IMIN_EDEVICE;
            kms += x;
        }
        stats->kernel_ms = kms;
    }
    return IMIN_OK;
}

int begin_call(imin_graph *g)
{
    if (!ok(hipSetDevice(g->device))) return IMIN_EDEVICE;
    g->kev_used = 0;
    g->small_auto_off = false;  // every call tries the wave kernel in its first round
    g->auto_pending = true;
    g->probe = 0;
    if (!ok(hipEventRecord(g->ev0, g->stream))) return IMIN_EDEVICE;
    return IMIN_OK;
}

void destroy(imin_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->batch_ms) {
        multi_free(*g->batch_ms);
        delete g->batch_ms;
        g->batch_ms = nullptr;
    }
    free_ws(g->main_ws);
    free_ws(g->big_ws);
    dfree(g->d_row_ptr);
    dfree(g->d_col4);
    dfree(g->d_edge);
    dfree(g->d_thr4);
    dfree(g->d_thr_orig);
    dfree(g->d_lo4);
    dfree(g->d_tl);
    dfree(g->d_in_ptr);
    dfree(g->d_in_edge);
    dfree(g->d_inelig);
    dfree(g->d_cand);
    dfree(g->d_seeds);
    dfree(g->d_list);
    dfree(g->d_D);
    dfree(g->d_stats);
    dfree(g->d_ctrl);
    dfree(g->d_sctrl);
    dfree(g->d_sj);
    dfree(g->d_inst);
    dfree(g->d_ovf);
    dfree(g->d_part_d);
    dfree(g->d_part_i);
    dfree(g->d_B);
    dfree(g->d_x);
    for (hipEvent_t e : g->kev) (void)hipEventDestroy(e);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

// A batched call runs every graph's work on one stream; each graph's own stream is put back
// when the call ends, however it ends.
struct StreamSwap {
    std::vector<std::pair<imin_graph *, hipStream_t>> saved;
    void use(imin_graph *g, hipStream_t s)
    {
        saved.emplace_back(g, g->stream);
        g->stream = s;
    }
    ~StreamSwap()
    {
        for (auto &p : saved) p.first->stream = p.second;
    }
};

// A device buffer of at least `count` elements, kept and grown only when too small.
template <class T>
bool grow(T *&p, size_t &cap, size_t count)
{
    count = std::max<size_t>(count, 1);
    if (p && cap >= count) return true;
    dfree(p);
    cap = 0;
    if (!ok(hipMalloc(&p, count * sizeof(T)))) {
        (void)hipGetLastError();
        return false;
    }
    cap = count;
    return true;
}

struct BatchItem {
    imin_instance *in = nullptr;
    imin_graph *g = nullptr;
    std::vector<int32_t> seeds;
    std::vector<uint32_t> inelig;
    std::vector<uint32_t> cand;  // GreedyReplace: CB
    int32_t rounds = 0;          // greedy rounds at most (GreedyReplace: 2k)
    int32_t nb = 0;              // blocker slots (GreedyReplace: k)
};

// A stream capture that is always ended, and the graph it made, released at scope exit.
struct GraphCapture {
    hipStream_t stream = nullptr;  // non-null while capturing
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int finish()
    {
        hipStream_t s = stream;
        stream = nullptr;
        if (!ok(hipStreamEndCapture(s, &graph)) ||
            !ok(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0))) {
            (void)hipGetLastError();
            return IMIN_EDEVICE;
        }
        return IMIN_OK;
    }
    ~GraphCapture()
    {
        if (stream) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

}  // namespace host
}  // namespace imin

using namespace imin::host;

extern "C" {

const char *imin_strerror(int status)
{
    switch (status) {
    case IMIN_OK: return "ok";
    case IMIN_EINVAL: return "invalid argument";
    case IMIN_ENOMEM: return "out of memory";
    case IMIN_EDEVICE: return "device error";
    case IMIN_ERANGE: return "size out of range";
    default: return "unknown status";
    }
}

int imin_graph_create(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                      const float *prob, imin_graph **out)
{
    return imin_graph_create_model(n, m, row_ptr, col, prob, IMIN_IC, out);
}

int imin_graph_create_model(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                            const float *prob, int model, imin_graph **out)
{
    if (!out || !row_ptr || n <= 0 || m < 0) return IMIN_EINVAL;
    if (model != IMIN_IC && model != IMIN_LT) return IMIN_EINVAL;
    if (n == INT32_MAX) return IMIN_ERANGE;
    if (row_ptr[0] != 0 || row_ptr[n] != m) return IMIN_EINVAL;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return IMIN_EINVAL;
    if (m > 0 && (!col || !prob)) return IMIN_EINVAL;
    for (int32_t e = 0; e < m; ++e) {
        if (col[e] < 0 || col[e] >= n) return IMIN_EINVAL;
        if (!(prob[e] >= 0.0f && prob[e] <= 1.0f)) return IMIN_EINVAL;  // rejects NaN
    }
    int ndev = 0;
    if (!ok(hipGetDeviceCount(&ndev)) || ndev <= 0) return IMIN_EDEVICE;

    imin_graph *g = new (std::nothrow) imin_graph();
    if (!g) return IMIN_ENOMEM;
    g->n = n;
    g->m = m;
    if (!ok(hipGetDevice(&g->device))) {
        delete g;
        return IMIN_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (!ok(hipGetDeviceProperties(&prop, g->device))) {
        delete g;
        return IMIN_EDEVICE;
    }
    g->num_cus = std::max(1, prop.multiProcessorCount);
    try {
        g->row_ptr.assign(row_ptr, row_ptr + n + 1);
        g->col.assign(col ? col : row_ptr, col ? col + m : row_ptr);
    } catch (...) {
        delete g;
        return IMIN_ENOMEM;
    }
    const int64_t quads = std::max<int64_t>(((int64_t)m + 3) / 4, 1);
    std::vector<uint32_t> hcol, hthr;
    try {
        hcol.assign((size_t)quads * 4, 0u);
        hthr.assign((size_t)quads * 4, 0u);  // padding edges have threshold 0: never live
    } catch (...) {
        delete g;
        return IMIN_ENOMEM;
    }
    for (int32_t e = 0; e < m; ++e) {
        hcol[(size_t)e] = (uint32_t)col[e];
        hthr[(size_t)e] = live_threshold(prob[e]);
    }
    // in-edge index: edge ids grouped by target, ascending (counting sort)
    std::vector<int32_t> in_ptr, in_edge;
    try {
        in_ptr.assign((size_t)n + 1, 0);
        in_edge.assign((size_t)std::max(m, 1), 0);
    } catch (...) {
        delete g;
        return IMIN_ENOMEM;
    }
    for (int32_t e = 0; e < m; ++e) ++in_ptr[(size_t)col[e] + 1];
    for (int32_t v = 0; v < n; ++v) in_ptr[(size_t)v + 1] += in_ptr[(size_t)v];
    {
        std::vector<int32_t> fill(in_ptr.begin(), in_ptr.end() - 1);
        for (int32_t e = 0; e < m; ++e) in_edge[(size_t)fill[(size_t)col[e]]++] = e;
    }
    // Linear-threshold model: the in-edges of v split [0, 2^24) into consecutive intervals,
    // edge k of v (ascending id) getting [bound_{k-1}, bound_k) with
    // bound_k = min(2^24, ceil(2^24 * (w_1 + ... + w_k))) from fp64 running sums.
    std::vector<uint32_t> hlo;
    if (model == IMIN_LT) {
        try {
            hlo.assign(hthr.size(), 0u);
        } catch (...) {
            delete g;
            return IMIN_ENOMEM;
        }
        for (int32_t v = 0; v < n; ++v) {
            double sum = 0.0;
            uint32_t prev = 0;
            for (int32_t k = in_ptr[(size_t)v]; k < in_ptr[(size_t)v + 1]; ++k) {
                const int32_t e = in_edge[(size_t)k];
                sum += (double)prob[e];
                const double bound = std::min(16777216.0, std::ceil(sum * 16777216.0));
                hlo[(size_t)e] = prev;
                hthr[(size_t)e] = (uint32_t)bound;
                prev = (uint32_t)bound;
            }
            if (sum > 1.0 + 1e-5) {
                delete g;
                return IMIN_EINVAL;
            }
        }
    }
    g->model = model;
    g->words = (n + 31) / 32;
    bool good =
        ok(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) &&
        ok(hipEventCreate(&g->ev0)) && ok(hipEventCreate(&g->ev1)) &&
        ok(hipMalloc(&g->d_row_ptr, (size_t)(n + 1) * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_col4, hcol.size() * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_thr4, hthr.size() * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_thr_orig, hthr.size() * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_in_ptr, in_ptr.size() * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_in_edge, in_edge.size() * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_inelig, (size_t)g->words * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_cand, (size_t)g->words * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_seeds, (size_t)n * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_list, 2 * (size_t)n * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_D, (size_t)n * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_stats, kStats * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_ctrl, imin::kCtrlWords * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_sctrl, 2 * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_inst, sizeof(imin::InstanceDesc))) &&
        ok(hipMalloc(&g->d_part_d, (size_t)g->parts * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_part_i, (size_t)g->parts * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_x, sizeof(int32_t))) &&
        (model != IMIN_LT || ok(hipMalloc(&g->d_lo4, hlo.size() * sizeof(uint32_t)))) &&
        (model != IMIN_LT || ok(hipMalloc(&g->d_tl, 2 * hlo.size() * sizeof(uint32_t)))) &&
        (model != IMIN_IC || ok(hipMalloc(&g->d_edge, hcol.size() * sizeof(uint4))));
    if (!good) {
        (void)hipGetLastError();
        destroy(g);
        return IMIN_ENOMEM;
    }
    if (!ok(hipMemcpy(g->d_row_ptr, row_ptr, (size_t)(n + 1) * sizeof(int32_t),
                      hipMemcpyHostToDevice)) ||
        !ok(hipMemcpy(g->d_col4, hcol.data(), hcol.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice)) ||
        !ok(hipMemcpy(g->d_thr4, hthr.data(), hthr.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice)) ||
        !ok(hipMemcpy(g->d_thr_orig, hthr.data(), hthr.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice)) ||
        !ok(hipMemcpy(g->d_in_ptr, in_ptr.data(), in_ptr.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice)) ||
        !ok(hipMemcpy(g->d_in_edge, in_edge.data(), in_edge.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice)) ||
        (model == IMIN_LT && !ok(hipMemcpy(g->d_lo4, hlo.data(), hlo.size() * sizeof(uint32_t),
                                           hipMemcpyHostToDevice)))) {
        destroy(g);
        return IMIN_EDEVICE;
    }
    if (model == IMIN_LT) {
        // per quad: its 4 targets, then its 4 lower bounds
        std::vector<uint32_t> htl;
        try {
            htl.assign(2 * hlo.size(), 0u);
        } catch (...) {
            destroy(g);
            return IMIN_ENOMEM;
        }
        for (size_t q = 0; q < hlo.size() / 4; ++q)
            for (int k = 0; k < 4; ++k) {
                htl[8 * q + k] = hcol[4 * q + k];
                htl[8 * q + 4 + k] = hlo[4 * q + k];
            }
        if (!ok(hipMemcpy(g->d_tl, htl.data(), htl.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice))) {
            destroy(g);
            return IMIN_EDEVICE;
        }
    }
    if (model == IMIN_IC) {
        // edge records: padding slots past m stay zero (their coins are never live)
        std::vector<uint4> hedge;
        try {
            hedge.assign(hcol.size(), make_uint4(0, 0, 0, 0));
        } catch (...) {
            destroy(g);
            return IMIN_ENOMEM;
        }
        for (int64_t e = 0; e < (int64_t)m; ++e) {
            const int32_t v = col[e];
            hedge[(size_t)e] = make_uint4((uint32_t)v, (uint32_t)row_ptr[v],
                                          (uint32_t)row_ptr[(size_t)v + 1], 0u);
        }
        if (!ok(hipMemcpy(g->d_edge, hedge.data(), hedge.size() * sizeof(uint4),
                          hipMemcpyHostToDevice))) {
            destroy(g);
            return IMIN_EDEVICE;
        }
    }
    *out = g;
    return IMIN_OK;
}

void imin_graph_destroy(imin_graph *g) { destroy(g); }

int imin_set_launch(imin_graph *g, int32_t slots, int64_t extra_cap)
{
    if (!g || slots < 0 || extra_cap < 0) return IMIN_EINVAL;
    if (slots > IMIN_MAX_SLOTS) return IMIN_ERANGE;
    g->force_slots = slots;
    g->force_xcap = extra_cap;
    return IMIN_OK;
}

}  // extern "C"

namespace {

// One Algorithm 2 call (counts != NULL) or a reachability-only estimate (counts == NULL).
int one_call(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
             uint32_t theta, uint64_t seed, uint64_t *counts, imin_stats *stats,
             int32_t *n_seeds)
{
    if (!g || theta == 0) return IMIN_EINVAL;
    if (theta > kMaxTheta) return IMIN_ERANGE;
    const bool reach_only = counts == nullptr;
    std::vector<int32_t> seeds;
    std::vector<uint32_t> inelig;
    int rc = seed_setup(g, S, nS, seeds, inelig);
    if (rc) return rc;
    if (blocked) {
        for (int32_t v = 0; v < g->n; ++v) {
            if (!blocked[v]) continue;
            // a seed cannot be blocked (Definition 2: B is a subset of V \ S)
            if (std::binary_search(seeds.begin(), seeds.end(), v)) return IMIN_EINVAL;
            inelig[v >> 5] |= 1u << (v & 31);
        }
    }
    rc = begin_call(g);
    if (rc) return rc;
    rc = prepare_workspaces(g);
    if (rc) return rc;
    rc = ensure_ovf(g, theta);
    if (rc) return rc;
    rc = ensure_sj(g, theta);
    if (rc) return rc;
    rc = upload_call_state(g, seeds, inelig, seed, theta);
    if (rc) return rc;
    rc = decrease_round(g, (int32_t)seeds.size(), theta, seed, 0, reach_only);
    if (rc) return rc;
    std::vector<unsigned long long> D;
    if (!reach_only) {
        D.resize((size_t)g->n);
        if (!ok(hipMemcpyAsync(D.data(), g->d_D, (size_t)g->n * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, g->stream)))
            return IMIN_EDEVICE;
    }
    imin_stats st;
    rc = finish_call(g, &st);
    if (rc) return rc;
    end_masks(g, {});
    if (!reach_only) std::memcpy(counts, D.data(), (size_t)g->n * sizeof(uint64_t));
    if (stats) *stats = st;
    *n_seeds = (int32_t)seeds.size();
    return IMIN_OK;
}

}  // namespace

extern "C" {

int imin_decrease(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                  uint32_t theta, uint64_t seed, uint64_t *counts, imin_stats *stats)
{
    if (!counts) return IMIN_EINVAL;
    int32_t ns = 0;
    return one_call(g, S, nS, blocked, theta, seed, counts, stats, &ns);
}

int imin_spread(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                uint32_t theta, uint64_t seed, double *spread, imin_stats *stats)
{
    if (!spread) return IMIN_EINVAL;
    imin_stats st;
    int32_t ns = 0;
    const int rc = one_call(g, S, nS, blocked, theta, seed, nullptr, &st, &ns);
    if (rc) return rc;
    *spread = (double)ns + (double)st.reached / (double)theta;
    if (stats) *stats = st;
    return IMIN_OK;
}

int imin_greedy(imin_graph *g, const int32_t *S, int32_t nS, int32_t b, uint32_t theta,
                uint64_t seed, int mode, int32_t *blockers, int32_t *n_blockers,
                imin_stats *stats)
{
    if (!g || theta == 0 || b < 0 || !n_blockers || (b > 0 && !blockers)) return IMIN_EINVAL;
    if (mode != IMIN_AG && mode != IMIN_GR) return IMIN_EINVAL;
    if (theta > kMaxTheta) return IMIN_ERANGE;
    std::vector<int32_t> seeds;
    std::vector<uint32_t> inelig;
    int rc = seed_setup(g, S, nS, seeds, inelig);
    if (rc) return rc;
    const int32_t ns = (int32_t)seeds.size();
    rc = begin_call(g);
    if (rc) return rc;
    rc = prepare_workspaces(g);
    if (rc) return rc;
    rc = ensure_ovf(g, theta);
    if (rc) return rc;
    rc = ensure_sj(g, theta);
    if (rc) return rc;
    rc = ensure_B(g, b);
    if (rc) return rc;
    rc = upload_call_state(g, seeds, inelig, seed, theta);
    if (rc) return rc;

    std::vector<int32_t> B;
    uint64_t call = 0;
    if (mode == IMIN_AG) {
        const int32_t rounds = std::min<int32_t>(b, g->n - ns);
        for (int32_t r = 0; r < rounds; ++r) {
            rc = decrease_round(g, ns, theta, seed, call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_inelig, 0, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, nullptr,
                                              g->d_B, r, g->d_x, thr_w(g), g->d_in_ptr,
                                              g->d_in_edge, g->stream)))
                return IMIN_EDEVICE;
        }
        B.assign((size_t)rounds, -1);
        if (rounds > 0 &&
            !ok(hipMemcpyAsync(B.data(), g->d_B, (size_t)rounds * sizeof(int32_t),
                               hipMemcpyDeviceToHost, g->stream)))
            return IMIN_EDEVICE;
    } else {
        // CB: out-neighbours of the merged seed, seeds excluded (Algorithm 4).
        std::vector<uint32_t> cand;
        const int32_t ncb = gr_candidates(g, seeds, inelig, cand);
        if (!ok(hipMemcpyAsync(g->d_cand, cand.data(), cand.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, g->stream)))
            return IMIN_EDEVICE;
        const int32_t k = std::min(ncb, b);
        for (int32_t r = 0; r < k; ++r) {
            rc = decrease_round(g, ns, theta, seed, call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_cand, 1, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, g->d_cand,
                                              g->d_B, r, g->d_x, thr_w(g), g->d_in_ptr,
                                              g->d_in_edge, g->stream)))
                return IMIN_EDEVICE;
        }
        B.assign((size_t)k, -1);
        if (k > 0) {
            if (!ok(hipMemcpyAsync(B.data(), g->d_B, (size_t)k * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, g->stream)) ||
                !ok(hipStreamSynchronize(g->stream)))
                return IMIN_EDEVICE;
        }
        for (int32_t v : B)
            if (v < 0) return IMIN_EDEVICE;
        const std::vector<int32_t> snapshot = B;
        for (int32_t i = k - 1; i >= 0; --i) {
            const int32_t u = snapshot[(size_t)i];
            const int32_t slot =
                (int32_t)(std::find(B.begin(), B.end(), u) - B.begin());
            if (!ok(imin::launch_set_bit(g->d_inelig, u, 0, g->stream)) ||
                !ok(imin::launch_mask_vertex(thr_w(g), reinterpret_cast<const uint32_t *>(
                                                           g->d_thr_orig),
                                             g->d_in_ptr, g->d_in_edge, u, nullptr, 1,
                                             g->stream)))
                return IMIN_EDEVICE;
            rc = decrease_round(g, ns, theta, seed, call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_inelig, 0, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, nullptr,
                                              g->d_B, slot, g->d_x, thr_w(g), g->d_in_ptr,
                                              g->d_in_edge, g->stream)))
                return IMIN_EDEVICE;
            int32_t x = -1;
            if (!ok(hipMemcpyAsync(&x, g->d_x, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   g->stream)) ||
                !ok(hipStreamSynchronize(g->stream)))
                return IMIN_EDEVICE;
            if (x < 0) return IMIN_EDEVICE;
            B[(size_t)slot] = x;
            if (x == u) break;
        }
    }
    imin_stats st;
    rc = finish_call(g, &st);
    if (rc) return rc;
    for (int32_t v : B)
        if (v < 0) return IMIN_EDEVICE;
    end_masks(g, B);
    std::copy(B.begin(), B.end(), blockers);
    *n_blockers = (int32_t)B.size();
    if (stats) *stats = st;
    return IMIN_OK;
}

int imin_set_small(imin_graph *g, int32_t enable, const imin_launch *launch)
{
    if (!g || enable < -1 || enable > 1 || !launch_ok(launch)) return IMIN_EINVAL;
    g->small_mode = enable;
    g->small_auto_off = false;
    g->small_launch = launch ? *launch : imin_launch{0, 0, 0, 0, 0};
    return IMIN_OK;
}

int imin_greedy_batch(imin_instance *inst, int32_t count, int mode, const imin_launch *launch)
{
    if (!inst || count <= 0 || (mode != IMIN_AG && mode != IMIN_GR) || !launch_ok(launch))
        return IMIN_EINVAL;
    const bool gr = mode == IMIN_GR;
    const imin_launch shape = launch ? *launch : imin_launch{0, 0, 0, 0, 0};
    std::vector<BatchItem> items((size_t)count);
    std::vector<imin_graph *> graphs;
    uint64_t theta_sum = 0;
    for (int32_t i = 0; i < count; ++i) {
        imin_instance &in = inst[i];
        if (!in.g || in.theta == 0 || in.b < 0 || !in.n_blockers || (in.b > 0 && !in.blockers))
            return IMIN_EINVAL;
        if (in.g->device != inst[0].g->device || in.g->model != inst[0].g->model)
            return IMIN_EINVAL;
        BatchItem &it = items[(size_t)i];
        it.in = &in;
        it.g = in.g;
        int rc = seed_setup(in.g, in.S, in.nS, it.seeds, it.inelig);
        if (rc) return rc;
        if (gr) {
            const int32_t k = std::min(gr_candidates(in.g, it.seeds, it.inelig, it.cand), in.b);
            it.nb = k;
            it.rounds = 2 * k;
        } else {
            it.rounds = std::min<int32_t>(in.b, in.g->n - (int32_t)it.seeds.size());
            it.nb = it.rounds;
        }
        theta_sum += in.theta;
        graphs.push_back(in.g);
    }
    std::sort(graphs.begin(), graphs.end());
    if (std::adjacent_find(graphs.begin(), graphs.end()) != graphs.end()) return IMIN_EINVAL;
    if (theta_sum > kMaxTheta) return IMIN_ERANGE;
    // Instances with more rounds first: the ones still active in round r form a prefix.
    std::stable_sort(items.begin(), items.end(),
                     [](const BatchItem &a, const BatchItem &b) { return a.rounds > b.rounds; });
    if (!ok(hipSetDevice(inst[0].g->device))) return IMIN_EDEVICE;
    for (imin_graph *g : graphs)
        if (!ok(hipStreamSynchronize(g->stream))) return IMIN_EDEVICE;
    const hipStream_t bs = inst[0].g->stream;
    StreamSwap swap;
    for (imin_graph *g : graphs) swap.use(g, bs);

    imin_graph *g0 = inst[0].g;
    g0->kev_used = 0;
    if (!ok(hipEventRecord(g0->ev0, bs))) return IMIN_EDEVICE;
    // Call state of every instance, staged in one buffer and put in place by one kernel.
    std::vector<imin::InstanceDesc> table((size_t)count);
    std::vector<imin::BatchStage> stages((size_t)count);
    std::vector<int32_t> stage, rounds((size_t)count);
    std::vector<uint32_t> prefix((size_t)count + 1, 0u);
    int32_t max_rounds = 0, max_nb = 0, gr_runs = 0;
    for (int32_t i = 0; i < count; ++i) {
        BatchItem &it = items[(size_t)i];
        imin_graph *g = it.g;
        const int rc = ensure_B(g, it.nb);
        if (rc) return rc;
        describe(g, (int32_t)it.seeds.size(), it.in->seed, it.in->theta);
        table[(size_t)i] = g->h_inst;
        table[(size_t)i].sample_base = prefix[(size_t)i];
        table[(size_t)i].gr_k = gr ? it.nb : -1;
        prefix[(size_t)i + 1] = prefix[(size_t)i] + it.in->theta;
        rounds[(size_t)i] = it.nb;  // blocker slots gathered at the end
        max_rounds = std::max(max_rounds, it.rounds);
        max_nb = std::max(max_nb, it.nb);
        if (gr && it.nb > 0) ++gr_runs;
        imin::BatchStage &S = stages[(size_t)i];
        S.seeds = (int64_t)stage.size();
        stage.insert(stage.end(), it.seeds.begin(), it.seeds.end());
        S.bits = (int64_t)stage.size();
        S.words = (int32_t)it.inelig.size();
        for (uint32_t w : it.inelig) stage.push_back((int32_t)w);
        S.prev = (int64_t)stage.size();
        S.nprev = g->mask_known ? (int32_t)g->masked.size() : -1;
        if (g->mask_known) stage.insert(stage.end(), g->masked.begin(), g->masked.end());
        g->mask_known = false;
        g->masked.clear();
        append_set_bits(it.inelig, g->masked);
        S.now = (int64_t)stage.size();
        S.nnow = (int32_t)g->masked.size();
        stage.insert(stage.end(), g->masked.begin(), g->masked.end());
        S.cand = -1;
        if (gr) {
            S.cand = (int64_t)stage.size();
            for (uint32_t w : it.cand) stage.push_back((int32_t)w);
        }
    }
    const int32_t stride = imin::kGatherB + std::max(max_nb, 1);
    int64_t max_n = 0, max_m = 0;
    for (const BatchItem &it : items) {
        max_n = std::max<int64_t>(max_n, it.g->n);
        max_m = std::max<int64_t>(max_m, it.g->m);
    }
    // The batch's scratch stays with its first graph for the next batch that graph leads
    // (same shape: nothing is allocated or cleared again).
    if (!g0->batch_ms) {
        g0->batch_ms = new (std::nothrow) MultiScratch();
        if (!g0->batch_ms) return IMIN_ENOMEM;
    }
    MultiScratch &ms = *g0->batch_ms;
    int rc = multi_alloc(ms, g0->num_cus, max_n, max_m, prefix[(size_t)count], count, bs);
    if (rc) {
        multi_free(ms);
        return rc;
    }
    if (!grow(ms.table, ms.table_cap, (size_t)count) ||
        !grow(ms.stages, ms.stages_cap, (size_t)count) ||
        !grow(ms.stage, ms.stage_cap, stage.size()) ||
        !grow(ms.rounds, ms.rounds_cap, (size_t)count) ||
        !grow(ms.out, ms.out_cap, (size_t)count * stride))
        return IMIN_ENOMEM;
    if (!ok(hipMemcpyAsync(ms.table, table.data(), table.size() * sizeof(imin::InstanceDesc),
                           hipMemcpyHostToDevice, bs)) ||
        !ok(hipMemcpyAsync(ms.stages, stages.data(), stages.size() * sizeof(imin::BatchStage),
                           hipMemcpyHostToDevice, bs)) ||
        !ok(hipMemcpyAsync(ms.stage, stage.data(), stage.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, bs)) ||
        !ok(hipMemcpyAsync(ms.rounds, rounds.data(), rounds.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, bs)) ||
        !ok(imin::launch_batch_setup(ms.table, ms.stages, ms.stage, count, bs)))
        return IMIN_EDEVICE;
    // Rounds: every launch is queued at once; nothing waits for the host until the end
    // (GreedyReplace: one word read back per round, the count of runs that have ended).
    const bool lt = g0->model == IMIN_LT;
    if (!ok(imin::launch_fill_u32(ms.ctrl + 9, 1, 0, bs))) return IMIN_EDEVICE;
    if (shape.graph && !gr) {
        // One HIP graph of kernel nodes for all rounds (slots clear their own maps when
        // their epochs wrap, so no memset is ever needed inside). Every kernel reads the
        // call's state through the device table, so the graph depends only on the launch
        // structure below; a call with the same structure replays the kept graph.
        std::vector<int64_t> key = {count, max_rounds, lt ? 1 : 0, g0->num_cus,
                                    shape.waves_per_cu, shape.quad_limit, shape.pick_div,
                                    shape.pack_per_cu, (int64_t)(uintptr_t)ms.table,
                                    (int64_t)(uintptr_t)ms.ctrl, (int64_t)(uintptr_t)ms.pi,
                                    (int64_t)(uintptr_t)ms.si, (int64_t)(uintptr_t)ms.oi,
                                    (int64_t)(uintptr_t)ms.part_d, (int64_t)ms.cap,
                                    (int64_t)(uintptr_t)ms.main_ws.map, ms.main_ws.slots,
                                    ms.main_ws.n, ms.main_ws.lcap, ms.main_ws.xcap,
                                    (int64_t)(uintptr_t)ms.big_ws.map, ms.big_ws.slots};
        {
            int32_t act = count;
            for (int32_t r = 0; r < max_rounds; ++r) {
                while (act > 0 && items[(size_t)act - 1].rounds <= r) --act;
                key.push_back(act);
                key.push_back(prefix[(size_t)act]);
            }
        }
        if (!ms.exec || ms.exec_key != key) {
            if (ms.exec) (void)hipGraphExecDestroy(ms.exec);
            ms.exec = nullptr;
            ms.exec_key.clear();
            GraphCapture cap;
            if (!ok(hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal)))
                return IMIN_EDEVICE;
            cap.stream = bs;
            int32_t act = count;
            for (int32_t r = 0; r < max_rounds; ++r) {
                while (act > 0 && items[(size_t)act - 1].rounds <= r) --act;
                rc = multi_round(ms, ms.table, act, prefix[(size_t)act], (uint32_t)r, shape,
                                 g0->num_cus, true, false, lt, bs);
                if (rc) return rc;
            }
            rc = cap.finish();
            if (rc) return rc;
            ms.exec = cap.exec;  // kept with the scratch
            cap.exec = nullptr;
            ms.exec_key = std::move(key);
        }
        hipEvent_t k0, k1;
        rc = kernel_events(g0, &k0, &k1);
        if (rc) return rc;
        if (!ok(hipEventRecord(k0, bs)) || !ok(hipGraphLaunch(ms.exec, bs)) ||
            !ok(hipEventRecord(k1, bs)))
            return IMIN_EDEVICE;
    } else {
        int32_t active = count;
        for (int32_t r = 0; r < max_rounds; ++r) {
            while (active > 0 && items[(size_t)active - 1].rounds <= r) --active;
            hipEvent_t k0, k1;
            rc = kernel_events(g0, &k0, &k1);
            if (rc) return rc;
            if (!ok(hipEventRecord(k0, bs))) return IMIN_EDEVICE;
            rc = multi_round(ms, ms.table, active, prefix[(size_t)active], (uint32_t)r,
                             shape, g0->num_cus, true, gr, lt, bs);
            if (rc) return rc;
            if (!ok(hipEventRecord(k1, bs))) return IMIN_EDEVICE;
            if (gr) {
                // every replacement pass that can still run has stopped: no more rounds
                uint32_t ended = 0;
                if (!ok(hipMemcpyAsync(&ended, ms.ctrl + 9, sizeof(ended), hipMemcpyDeviceToHost,
                                       bs)) ||
                    !ok(hipStreamSynchronize(bs)))
                    return IMIN_EDEVICE;
                if ((int32_t)ended >= gr_runs) break;
            }
        }
    }
    // Results: every graph's blocker slots, counters and error flag, gathered into one
    // buffer, then one copy and one wait.
    std::vector<int32_t> out((size_t)count * stride);
    if (!ok(imin::launch_batch_gather(ms.table, ms.rounds, ms.out, stride, count, bs)) ||
        !ok(hipMemcpyAsync(out.data(), ms.out, out.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, bs)) ||
        !ok(hipEventRecord(g0->ev1, bs)) || !ok(hipEventSynchronize(g0->ev1)))
        return IMIN_EDEVICE;
    uint32_t wave_err = 0, wg_err = 0;
    rc = multi_errors(ms, &wave_err, &wg_err, bs);
    if (rc) return rc;
    if (wave_err || wg_err) return IMIN_EDEVICE;
    std::vector<std::vector<int32_t>> B((size_t)count);
    std::vector<std::array<unsigned long long, kStats>> st((size_t)count);
    std::vector<uint32_t> err((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const int32_t *o = out.data() + (size_t)i * stride;
        for (int k = 0; k < kStats; ++k)
            st[(size_t)i][k] = (unsigned long long)(uint32_t)o[2 * k] |
                               ((unsigned long long)(uint32_t)o[2 * k + 1] << 32);
        err[(size_t)i] = (uint32_t)o[imin::kGatherErr];
        B[(size_t)i].assign(o + imin::kGatherB, o + imin::kGatherB + items[(size_t)i].nb);
    }
    float total_ms = 0.0f;
    if (!ok(hipEventElapsedTime(&total_ms, g0->ev0, g0->ev1))) return IMIN_EDEVICE;
    double kms = 0.0;
    for (size_t k = 0; k + 1 < g0->kev_used; k += 2) {
        float x = 0.0f;
        if (!ok(hipEventElapsedTime(&x, g0->kev[k], g0->kev[k + 1]))) return IMIN_EDEVICE;
        kms += x;
    }
    for (int32_t i = 0; i < count; ++i) {
        if (err[(size_t)i] != 0) return IMIN_EDEVICE;
        for (int32_t v : B[(size_t)i])
            if (v < 0) return IMIN_EDEVICE;
    }
    for (int32_t i = 0; i < count; ++i) {
        BatchItem &it = items[(size_t)i];
        end_masks(it.g, B[(size_t)i]);
        std::copy(B[(size_t)i].begin(), B[(size_t)i].end(), it.in->blockers);
        *it.in->n_blockers = it.nb;
        if (it.in->stats) {
            imin_stats &o = *it.in->stats;
            o.samples = st[(size_t)i][0];
            o.reached = st[(size_t)i][1];
            o.edges_scanned = st[(size_t)i][2];
            o.live_edges = st[(size_t)i][3];
            o.spilled = st[(size_t)i][4];
            o.wave_samples = st[(size_t)i][5];
            o.pack_samples = st[(size_t)i][6];
            o.device_ms = total_ms;
            o.kernel_ms = kms;
        }
    }
    return IMIN_OK;
}

}  // extern "C"
