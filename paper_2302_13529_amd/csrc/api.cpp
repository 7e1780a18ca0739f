// api.cpp -- host side of libimin: validation, device residency of the graph, scratch
// sizing, and the greedy drivers (Algorithms 3 and 4 of arXiv 2302.13529) as device-side
// round loops. Every step of the estimate runs in the kernels of decrease.hip/select.hip.
#include "imin.h"
#include "imin_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using imin::DecreaseArgs;
using imin::Workspace;

struct imin_graph {
    int device = 0;
    int32_t n = 0;
    int32_t m = 0;
    int num_cus = 1;
    std::vector<int32_t> row_ptr;  // host copies: out-neighbours of the seeds (GR)
    std::vector<int32_t> col;
    int32_t *d_row_ptr = nullptr;
    uint4 *d_col4 = nullptr;   // edge targets, 4 per quad, padded to a whole quad
    uint4 *d_thr4 = nullptr;   // live thresholds, same layout
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t words = 0;                       // 32-bit words of a vertex bitmap
    uint32_t *d_inelig = nullptr;            // seeds and blocked vertices
    uint32_t *d_cand = nullptr;              // GR candidate set CB
    int32_t *d_seeds = nullptr;              // distinct seeds (capacity n)
    unsigned long long *d_D = nullptr;       // n
    unsigned long long *d_stats = nullptr;   // 5: samples, reached, scanned, live, spilled
    uint32_t *d_ctrl = nullptr;              // 4: next main, next spill, spill count, error
    uint32_t *d_ovf = nullptr;
    uint32_t ovf_cap = 0;
    unsigned long long *d_part_d = nullptr;
    int32_t *d_part_i = nullptr;
    int32_t parts = 4096;
    int32_t *d_B = nullptr;
    int32_t B_cap = 0;
    int32_t *d_x = nullptr;
    Workspace main_ws, big_ws;
    std::vector<int32_t> marked;   // vertices stamped kInelig in every slot map
    bool marks_valid = true;       // false after a call that stopped half-way
    int32_t *d_list = nullptr;     // n: vertex lists for stamping
    std::vector<hipEvent_t> kev;  // pairs around each decrease launch of the current call
    size_t kev_used = 0;
    int32_t force_slots = 0;
    int64_t force_xcap = 0;
};

namespace {

constexpr uint32_t kSpillSlots = 2;
// The per-launch work counter is 32-bit and every workgroup takes one index past the end.
constexpr uint32_t kMaxTheta = 1u << 31;

bool ok(hipError_t e) { return e == hipSuccess; }

// ceil(p * 2^24) for p in [0, 1]; the product by a power of two is exact in fp32.
uint32_t live_threshold(float p)
{
    if (p <= 0.0f) return 0u;
    if (p >= 1.0f) return 1u << 24;
    return (uint32_t)std::ceil(p * 16777216.0f);
}

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_ws(Workspace &ws)
{
    dfree(ws.map);
    dfree(ws.loc);
    dfree(ws.lvl);
    dfree(ws.extra);
    dfree(ws.epoch);
    ws = Workspace();
}

size_t slot_bytes(int64_t n, int64_t lcap, int64_t xcap)
{
    return (size_t)n * sizeof(imin::SlotEntry) + (size_t)lcap * sizeof(imin::LocalVtx) +
           (size_t)(lcap + 1) * sizeof(int32_t) + (size_t)xcap * sizeof(int2) + sizeof(uint32_t);
}

int alloc_ws(imin_graph *g, Workspace &ws, int32_t slots, int64_t lcap, int64_t xcap)
{
    if (ws.slots == slots && ws.lcap == lcap && ws.xcap == xcap) return IMIN_OK;
    free_ws(ws);
    const size_t S = (size_t)slots;
    bool good = ok(hipMalloc(&ws.map, S * (size_t)g->n * sizeof(imin::SlotEntry))) &&
                ok(hipMalloc(&ws.loc, S * (size_t)lcap * sizeof(imin::LocalVtx))) &&
                ok(hipMalloc(&ws.lvl, S * (size_t)(lcap + 1) * sizeof(int32_t))) &&
                ok(hipMalloc(&ws.extra, S * (size_t)std::max<int64_t>(xcap, 1) * sizeof(int2))) &&
                ok(hipMalloc(&ws.epoch, S * sizeof(uint32_t)));
    if (!good) {
        free_ws(ws);
        (void)hipGetLastError();
        return IMIN_ENOMEM;
    }
    if (!ok(hipMemsetAsync(ws.map, 0, S * (size_t)g->n * sizeof(imin::SlotEntry), g->stream)) ||
        !ok(hipMemsetAsync(ws.epoch, 0, S * sizeof(uint32_t), g->stream))) {
        free_ws(ws);
        return IMIN_EDEVICE;
    }
    ws.slots = slots;
    ws.lcap = lcap;
    ws.xcap = xcap;
    ws.epochs_used = 0;
    ws.bytes = S * slot_bytes(g->n, lcap, xcap);
    return IMIN_OK;
}

// Per-slot scratch: every local array holds all n vertices plus the root, so only the
// extra-edge list can overflow. Its default capacity covers a quarter of the vertices; a
// graph whose m is below that can never overflow and needs no spill path.
int prepare_workspaces(imin_graph *g)
{
    if (!g->marks_valid) {
        free_ws(g->main_ws);
        free_ws(g->big_ws);
        g->marked.clear();
        g->marks_valid = true;
    }
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
        const size_t per = slot_bytes(g->n, lcap, xcap);
        const size_t by_mem = std::max<size_t>(1, (free_b / 2) / per);
        slots = (int32_t)std::min<size_t>((size_t)2 * g->num_cus, by_mem);
        if (g->main_ws.slots > 0 && g->main_ws.lcap == lcap && g->main_ws.xcap == xcap &&
            g->main_ws.slots <= slots)
            slots = g->main_ws.slots;  // keep a working allocation
    }
    int rc = alloc_ws(g, g->main_ws, slots, lcap, xcap);
    if (rc) return rc;
    if (xcap < xmax) {
        rc = alloc_ws(g, g->big_ws, kSpillSlots, lcap, xmax);
        if (rc) return rc;
    } else {
        free_ws(g->big_ws);
    }
    return IMIN_OK;
}

// Keep every slot's 32-bit epoch from wrapping: a launch of theta samples raises any slot's
// epoch by at most theta.
int guard_epochs(imin_graph *g, Workspace &ws, uint32_t theta)
{
    if (ws.slots == 0) return IMIN_OK;
    if (ws.epochs_used + theta + 1 < 0xFFFFFFFFull) {
        ws.epochs_used += theta;
        return IMIN_OK;
    }
    if (!ok(hipMemsetAsync(ws.map, 0, (size_t)ws.slots * g->n * sizeof(imin::SlotEntry),
                           g->stream)) ||
        !ok(hipMemsetAsync(ws.epoch, 0, (size_t)ws.slots * sizeof(uint32_t), g->stream)) ||
        !ok(imin::launch_mark_bitmap(ws.map, ws.slots, g->n, g->d_inelig, g->stream)))
        return IMIN_EDEVICE;
    ws.epochs_used = theta;
    return IMIN_OK;
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

int upload_call_state(imin_graph *g, const std::vector<int32_t> &seeds,
                      const std::vector<uint32_t> &inelig)
{
    if (!ok(hipMemcpyAsync(g->d_seeds, seeds.data(), seeds.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, g->stream)) ||
        !ok(hipMemcpyAsync(g->d_inelig, inelig.data(), inelig.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, g->stream)))
        return IMIN_EDEVICE;
    if (!ok(imin::launch_fill_u64(g->d_stats, 5, 0, g->stream)) ||
        !ok(imin::launch_fill_u32(g->d_ctrl, 4, 0, g->stream)))
        return IMIN_EDEVICE;
    // Slot-map stamps: clear the previous call's seeds and blockers, stamp the new ones.
    Workspace *wss[2] = {&g->main_ws, &g->big_ws};
    g->marks_valid = false;
    for (Workspace *ws : wss) {
        if (ws->slots == 0) continue;
        if (!g->marked.empty()) {
            if (!ok(hipMemcpyAsync(g->d_list, g->marked.data(), g->marked.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, g->stream)) ||
                !ok(imin::launch_set_stamps(ws->map, ws->slots, g->n, g->d_list,
                                            (int32_t)g->marked.size(), 0u, g->stream)))
                return IMIN_EDEVICE;
        }
        if (!ok(imin::launch_mark_bitmap(ws->map, ws->slots, g->n, g->d_inelig, g->stream)))
            return IMIN_EDEVICE;
    }
    g->marked.clear();
    for (int32_t v = 0; v < g->n; ++v)
        if ((inelig[v >> 5] >> (v & 31)) & 1u) g->marked.push_back(v);
    return IMIN_OK;
}

// A vertex joins (value kInelig) or leaves (value 0) the seed/blocked stamps of all slots;
// v_dev, when non-null, holds the vertex id on the device.
int stamp_vertex(imin_graph *g, int32_t v, const int32_t *v_dev, uint32_t value)
{
    Workspace *wss[2] = {&g->main_ws, &g->big_ws};
    for (Workspace *ws : wss)
        if (!ok(imin::launch_set_stamp(ws->map, ws->slots, g->n, v, v_dev, value, g->stream)))
            return IMIN_EDEVICE;
    return IMIN_OK;
}

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

// One call of Algorithm 2 with Philox key `key`, leaving D on the device.
int decrease_round(imin_graph *g, int32_t nseeds, uint32_t theta, uint64_t key)
{
    int rc = guard_epochs(g, g->main_ws, theta);
    if (rc) return rc;
    const bool spill = g->big_ws.slots > 0;
    if (spill) {
        rc = guard_epochs(g, g->big_ws, theta);
        if (rc) return rc;
    }
    if (!ok(imin::launch_fill_u64(g->d_D, g->n, 0, g->stream)) ||
        !ok(imin::launch_fill_u32(g->d_ctrl, 3, 0, g->stream)))
        return IMIN_EDEVICE;
    DecreaseArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->d_row_ptr;
    a.col4 = g->d_col4;
    a.thr4 = g->d_thr4;
    a.seeds = g->d_seeds;
    a.nseeds = nseeds;
    a.n = g->n;
    a.key_lo = (uint32_t)key;
    a.key_hi = (uint32_t)(key >> 32);
    a.theta = theta;
    a.sample_list = nullptr;
    a.sample_count = nullptr;
    a.next = g->d_ctrl + 0;
    a.D = g->d_D;
    a.stats = g->d_stats;
    a.ovf_list = g->d_ovf;
    a.ovf_count = g->d_ctrl + 2;
    a.error = g->d_ctrl + 3;
    a.spill_ok = spill ? 1 : 0;
    a.ws = g->main_ws;
    a.ws.slots = (int32_t)std::min<uint32_t>((uint32_t)g->main_ws.slots, theta);
    hipEvent_t k0, k1;
    rc = kernel_events(g, &k0, &k1);
    if (rc) return rc;
    if (!ok(hipEventRecord(k0, g->stream))) return IMIN_EDEVICE;
    if (!ok(imin::launch_decrease(a, g->stream))) return IMIN_EDEVICE;
    if (spill) {
        a.sample_list = g->d_ovf;
        a.sample_count = g->d_ctrl + 2;
        a.next = g->d_ctrl + 1;
        a.spill_ok = 0;
        a.ws = g->big_ws;
        if (!ok(imin::launch_decrease(a, g->stream))) return IMIN_EDEVICE;
    }
    if (!ok(hipEventRecord(k1, g->stream))) return IMIN_EDEVICE;
    return IMIN_OK;
}

// Copies the stats and the error flag back; returns IMIN_EDEVICE if a sample was lost.
int finish_call(imin_graph *g, imin_stats *stats)
{
    unsigned long long st[5];
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
    if (!ok(hipEventRecord(g->ev0, g->stream))) return IMIN_EDEVICE;
    return IMIN_OK;
}

void destroy(imin_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    free_ws(g->main_ws);
    free_ws(g->big_ws);
    dfree(g->d_row_ptr);
    dfree(g->d_col4);
    dfree(g->d_thr4);
    dfree(g->d_inelig);
    dfree(g->d_cand);
    dfree(g->d_seeds);
    dfree(g->d_list);
    dfree(g->d_D);
    dfree(g->d_stats);
    dfree(g->d_ctrl);
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

}  // namespace

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
    if (!out || !row_ptr || n <= 0 || m < 0) return IMIN_EINVAL;
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
    g->words = (n + 31) / 32;
    bool good =
        ok(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) &&
        ok(hipEventCreate(&g->ev0)) && ok(hipEventCreate(&g->ev1)) &&
        ok(hipMalloc(&g->d_row_ptr, (size_t)(n + 1) * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_col4, hcol.size() * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_thr4, hthr.size() * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_inelig, (size_t)g->words * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_cand, (size_t)g->words * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_seeds, (size_t)n * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_list, (size_t)n * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_D, (size_t)n * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_stats, 5 * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_ctrl, 4 * sizeof(uint32_t))) &&
        ok(hipMalloc(&g->d_part_d, (size_t)g->parts * sizeof(unsigned long long))) &&
        ok(hipMalloc(&g->d_part_i, (size_t)g->parts * sizeof(int32_t))) &&
        ok(hipMalloc(&g->d_x, sizeof(int32_t)));
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
                      hipMemcpyHostToDevice))) {
        destroy(g);
        return IMIN_EDEVICE;
    }
    *out = g;
    return IMIN_OK;
}

void imin_graph_destroy(imin_graph *g) { destroy(g); }

int imin_set_launch(imin_graph *g, int32_t slots, int64_t extra_cap)
{
    if (!g || slots < 0 || extra_cap < 0) return IMIN_EINVAL;
    g->force_slots = slots;
    g->force_xcap = extra_cap;
    return IMIN_OK;
}

int imin_decrease(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                  uint32_t theta, uint64_t seed, uint64_t *counts, imin_stats *stats)
{
    if (!g || !counts || theta == 0) return IMIN_EINVAL;
    if (theta > kMaxTheta) return IMIN_ERANGE;
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
    rc = upload_call_state(g, seeds, inelig);
    if (rc) return rc;
    rc = decrease_round(g, (int32_t)seeds.size(), theta, seed);
    if (rc) return rc;
    std::vector<unsigned long long> D((size_t)g->n);
    if (!ok(hipMemcpyAsync(D.data(), g->d_D, (size_t)g->n * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, g->stream)))
        return IMIN_EDEVICE;
    imin_stats st;
    rc = finish_call(g, &st);
    if (rc) return rc;
    g->marks_valid = true;
    std::memcpy(counts, D.data(), (size_t)g->n * sizeof(uint64_t));
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
    rc = ensure_B(g, b);
    if (rc) return rc;
    rc = upload_call_state(g, seeds, inelig);
    if (rc) return rc;

    std::vector<int32_t> B;
    uint64_t call = 0;
    if (mode == IMIN_AG) {
        const int32_t rounds = std::min<int32_t>(b, g->n - ns);
        for (int32_t r = 0; r < rounds; ++r) {
            rc = decrease_round(g, ns, theta, seed + call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_inelig, 0, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, nullptr,
                                              g->d_B, r, g->d_x, g->stream)))
                return IMIN_EDEVICE;
            rc = stamp_vertex(g, 0, g->d_x, imin::kInelig);
            if (rc) return rc;
        }
        B.assign((size_t)rounds, -1);
        if (rounds > 0 &&
            !ok(hipMemcpyAsync(B.data(), g->d_B, (size_t)rounds * sizeof(int32_t),
                               hipMemcpyDeviceToHost, g->stream)))
            return IMIN_EDEVICE;
    } else {
        // CB: out-neighbours of the merged seed, seeds excluded (Algorithm 4, line 1).
        std::vector<uint32_t> cand((size_t)g->words, 0u);
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
        if (!ok(hipMemcpyAsync(g->d_cand, cand.data(), cand.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, g->stream)))
            return IMIN_EDEVICE;
        const int32_t k = std::min(ncb, b);
        for (int32_t r = 0; r < k; ++r) {
            rc = decrease_round(g, ns, theta, seed + call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_cand, 1, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, g->d_cand,
                                              g->d_B, r, g->d_x, g->stream)))
                return IMIN_EDEVICE;
            rc = stamp_vertex(g, 0, g->d_x, imin::kInelig);
            if (rc) return rc;
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
            if (!ok(imin::launch_set_bit(g->d_inelig, u, 0, g->stream))) return IMIN_EDEVICE;
            rc = stamp_vertex(g, u, nullptr, 0u);
            if (rc) return rc;
            rc = decrease_round(g, ns, theta, seed + call);
            if (rc) return rc;
            ++call;
            if (!ok(imin::launch_argmax_apply(g->d_D, g->d_inelig, 0, g->n, g->d_part_d,
                                              g->d_part_i, g->parts, g->d_inelig, nullptr,
                                              g->d_B, slot, g->d_x, g->stream)))
                return IMIN_EDEVICE;
            rc = stamp_vertex(g, 0, g->d_x, imin::kInelig);
            if (rc) return rc;
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
    // the stamped set is now the seeds plus the final blockers
    for (int32_t v : B) g->marked.push_back(v);
    g->marks_valid = true;
    std::copy(B.begin(), B.end(), blockers);
    *n_blockers = (int32_t)B.size();
    if (stats) *stats = st;
    return IMIN_OK;
}

}  // extern "C"
