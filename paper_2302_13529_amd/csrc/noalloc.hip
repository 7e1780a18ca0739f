// noalloc.hip -- imin_decrease_noalloc: Algorithm 2 of arXiv 2302.13529 (the same counts as
// imin_decrease) for callers that cannot allocate device memory: code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation.
//
// Every scratch buffer of the call -- the seed staging, the blocked marks, the wave kernel's
// hand-over list, the workgroup kernel's slot maps, local records, level starts and extra-edge
// lists, its overflow list and the large-capacity spill slots -- is carved from one
// file-scope device array of kScratchBytes per GPU. The caller passes the graph (made
// resident by imin_graph_create), the host seed set and blocked marks, and a device buffer of
// n uint64 counts, which the kernels write directly. No hipMalloc, hipFree or other
// allocating routine is called.
#include "graph.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // IMIN_NOALLOC_SCRATCH_BYTES

// The scratch array. In host code this name stands for the symbol, not for a device
// address: host code only ever uses the per-device address that hipGetSymbolAddress returns.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev`, looked up once per device.
int scratch_on(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return IMIN_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return IMIN_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return IMIN_OK;
}

constexpr int kBlock = 256;

// Distinct seeds: the first thread to set a seed's bit appends it (any order; the counts do
// not depend on the order of the seed list).
__global__ void seed_set_kernel(const int32_t *S, int32_t nS, uint32_t *bits, int32_t *out,
                                uint32_t *count)
{
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < nS; i += gridDim.x * kBlock) {
        const int32_t s = S[i];
        const uint32_t bit = 1u << (s & 31);
        if (!(atomicOr(&bits[s >> 5], bit) & bit)) out[atomicAdd(count, 1u)] = s;
    }
}

// In-edge thresholds of every vertex v with marks[v] != 0: 0, or restored from orig.
__global__ void mask_marked_kernel(uint32_t *thr, const uint32_t *orig, const int32_t *in_ptr,
                                   const int32_t *in_edge, const uint8_t *marks, int32_t n,
                                   int restore)
{
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        if (!marks[v]) continue;
        for (int32_t k = in_ptr[v]; k < in_ptr[v + 1]; ++k) {
            const int32_t e = in_edge[k];
            thr[e] = restore ? orig[e] : 0u;
        }
    }
}

int grid_of(int64_t count)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (count + kBlock - 1) / kBlock));
}

// A bump allocator over the scratch array (offsets only; nothing is allocated).
struct Carve {
    unsigned char *base;
    size_t used = 0;
    bool fits = true;
    template <class T>
    T *take(size_t count)
    {
        const size_t off = (used + 255) & ~size_t(255);
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (off + bytes > kScratchBytes) {
            fits = false;
            return nullptr;
        }
        used = off + bytes;
        return reinterpret_cast<T *>(base + off);
    }
};

// Slot-major workgroup-kernel scratch of `slots` slots in the carve.
bool carve_ws(Carve &c, imin::Workspace &ws, int64_t n, int32_t slots, int64_t lcap, int64_t xcap,
              bool rng)
{
    int32_t lbits = 1;
    while (lbits < 32 && (int64_t(1) << lbits) <= lcap) ++lbits;
    if (lbits > 31) return false;
    const size_t S = (size_t)slots;
    ws.map = c.take<unsigned long long>(S * (size_t)n);
    ws.loc = c.take<imin::LocalVtx>(S * (size_t)lcap);
    ws.lvl = c.take<int32_t>(S * (size_t)(lcap + 1));
    ws.extra = c.take<int2>(S * (size_t)std::max<int64_t>(xcap, 1));
    ws.epoch = c.take<uint32_t>(S);
    ws.dirty = c.take<uint32_t>(S);
    ws.rng = rng ? c.take<int2>(S * (size_t)lcap) : nullptr;
    ws.slots = slots;
    ws.n = n;
    ws.lcap = lcap;
    ws.xcap = xcap;
    ws.lbits = lbits;
    return c.fits;
}

}  // namespace

using namespace imin::host;

extern "C" {

int imin_decrease_noalloc(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                          uint32_t theta, uint64_t seed, uint64_t *d_counts, imin_stats *stats)
{
    if (!g || !S || nS <= 0 || theta == 0 || !d_counts) return IMIN_EINVAL;
    if (theta > kMaxTheta) return IMIN_ERANGE;
    for (int32_t i = 0; i < nS; ++i) {
        if (S[i] < 0 || S[i] >= g->n) return IMIN_EINVAL;
        if (blocked && blocked[S[i]]) return IMIN_EINVAL;  // B is a subset of V \ S
    }
    if (!ok(hipSetDevice(g->device))) return IMIN_EDEVICE;
    unsigned char *base = nullptr;
    int rc = scratch_on(g->device, &base);
    if (rc) return rc;

    // Layout of this call's scratch.
    const int64_t n = g->n, m = g->m;
    const int64_t lcap = n + 1, xmax = m + 1;
    const int64_t xcap = std::min<int64_t>(std::max<int64_t>(4096, lcap / 4), xmax);
    Carve c{base};
    uint32_t *bits = c.take<uint32_t>((size_t)g->words);
    int32_t *s_in = c.take<int32_t>((size_t)nS);
    int32_t *s_set = c.take<int32_t>((size_t)nS);
    uint32_t *s_count = c.take<uint32_t>(1);
    uint8_t *marks = blocked ? c.take<uint8_t>((size_t)n) : nullptr;
    uint32_t *sj = c.take<uint32_t>(theta);
    uint32_t *ovf = c.take<uint32_t>(theta);
    // independent cascade: slots keep each claimed vertex's row range
    const bool rng = g->model == IMIN_IC;
    imin::Workspace big_ws;
    if (xcap < xmax && !carve_ws(c, big_ws, n, 2, lcap, xmax, rng)) return IMIN_ERANGE;
    if (!c.fits) return IMIN_ERANGE;
    const size_t fixed = c.used;
    // as many workgroup slots as the rest holds, up to the usual count
    Carve probe{base, fixed};
    imin::Workspace one;
    if (!carve_ws(probe, one, n, 1, lcap, xcap, rng)) return IMIN_ERANGE;
    const size_t per_slot = probe.used - fixed + 7 * 256;
    const int32_t slots = (int32_t)std::max<size_t>(
        1, std::min<size_t>((size_t)imin::kSlotsPerCu * g->num_cus,
                            (kScratchBytes - fixed) / per_slot));
    imin::Workspace main_ws;
    if (!carve_ws(c, main_ws, n, slots, lcap, xcap, rng)) return IMIN_ERANGE;
    if (xcap >= xmax) big_ws = imin::Workspace();

    hipStream_t st = g->stream;
    uint32_t *thr = reinterpret_cast<uint32_t *>(g->d_thr4);
    const uint32_t *orig = reinterpret_cast<const uint32_t *>(g->d_thr_orig);
    // Thresholds: undo what an earlier call on this graph left masked; from here until the
    // end of the call the graph's masking state is unknown to the other entry points.
    if (!g->mask_known) {
        const int64_t quads = std::max<int64_t>((m + 3) / 4, 1);
        if (!ok(hipMemcpyAsync(g->d_thr4, g->d_thr_orig, (size_t)quads * sizeof(uint4),
                               hipMemcpyDeviceToDevice, st)))
            return IMIN_EDEVICE;
    } else if (!g->masked.empty()) {
        if (!ok(hipMemcpyAsync(g->d_list, g->masked.data(), g->masked.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, st)) ||
            !ok(imin::launch_mask_list(thr, orig, g->d_in_ptr, g->d_in_edge, g->d_list,
                                       (int32_t)g->masked.size(), 1, st)))
            return IMIN_EDEVICE;
    }
    g->masked.clear();
    g->mask_known = false;

    // Distinct seeds, blocked marks, cleared counters and slot maps.
    uint32_t nseeds = 0;
    if (!ok(imin::launch_fill_u32(bits, g->words, 0u, st)) ||
        !ok(imin::launch_fill_u32(s_count, 1, 0u, st)) ||
        !ok(hipMemcpyAsync(s_in, S, (size_t)nS * sizeof(int32_t), hipMemcpyHostToDevice, st)) ||
        (blocked && !ok(hipMemcpyAsync(marks, blocked, (size_t)n, hipMemcpyHostToDevice, st))))
        return IMIN_EDEVICE;
    hipLaunchKernelGGL(seed_set_kernel, dim3(grid_of(nS)), dim3(kBlock), 0, st, s_in, nS, bits,
                       s_set, s_count);
    if (!ok(hipGetLastError()) ||
        !ok(hipMemcpyAsync(&nseeds, s_count, sizeof(nseeds), hipMemcpyDeviceToHost, st)) ||
        !ok(hipStreamSynchronize(st)))
        return IMIN_EDEVICE;
    if (!ok(imin::launch_mask_list(thr, orig, g->d_in_ptr, g->d_in_edge, s_set, (int32_t)nseeds,
                                   0, st)))
        return IMIN_EDEVICE;
    if (blocked) {
        hipLaunchKernelGGL(mask_marked_kernel, dim3(grid_of(n)), dim3(kBlock), 0, st, thr, orig,
                           g->d_in_ptr, g->d_in_edge, marks, (int32_t)n, 0);
        if (!ok(hipGetLastError())) return IMIN_EDEVICE;
    }
    const imin::Workspace *wss[2] = {&main_ws, &big_ws};
    for (const imin::Workspace *w : wss) {
        if (w->slots <= 0) continue;
        if (!ok(imin::launch_fill_u32(reinterpret_cast<uint32_t *>(w->map),
                                      2 * (int64_t)w->slots * w->n, 0u, st)) ||
            !ok(imin::launch_fill_u32(w->epoch, w->slots, 0u, st)) ||
            !ok(imin::launch_fill_u32(w->dirty, w->slots, 0u, st)))
            return IMIN_EDEVICE;
    }
    if (!ok(imin::launch_fill_u64(reinterpret_cast<unsigned long long *>(d_counts), n, 0ull, st)) ||
        !ok(imin::launch_fill_u64(g->d_stats, kStats, 0ull, st)) ||
        !ok(imin::launch_fill_u32(g->d_ctrl, imin::kCtrlWords, 0u, st)) ||
        !ok(imin::launch_fill_u32(g->d_sctrl, 2, 0u, st)))
        return IMIN_EDEVICE;

    // The graph as the one instance of the wave kernel, counting into the caller's buffer.
    imin::InstanceDesc I{};
    I.row_ptr = g->d_row_ptr;
    I.col4 = g->d_col4;
    I.edge = g->d_edge;
    I.thr4 = g->d_thr4;
    I.lo4 = g->d_lo4;
    I.tl = g->d_tl;
    I.in_ptr = g->d_in_ptr;
    I.in_edge = g->d_in_edge;
    I.inelig = bits;
    I.seeds = s_set;
    I.D = reinterpret_cast<unsigned long long *>(d_counts);
    I.stats = g->d_stats;
    I.thr_orig = g->d_thr_orig;
    I.ctrl = g->d_ctrl;
    I.nseeds = (int32_t)nseeds;
    I.n = g->n;
    I.nquads = (int32_t)std::max<int64_t>((m + 3) / 4, 1);
    I.seed_lo = (uint32_t)seed;
    I.seed_hi = (uint32_t)(seed >> 32);
    I.theta = theta;
    I.sample_base = 0;
    if (!ok(hipEventRecord(g->ev0, st)) ||
        !ok(hipMemcpyAsync(g->d_inst, &I, sizeof(I), hipMemcpyHostToDevice, st)))
        return IMIN_EDEVICE;
    imin::SmallArgs s;
    std::memset(&s, 0, sizeof(s));
    s.inst = g->d_inst;
    s.ninst = 1;
    s.total = theta;
    s.round = 0;
    small_shape(s, g->small_launch);
    s.lt = g->model == IMIN_LT ? 1 : 0;
    s.next = g->d_sctrl + 0;
    s.spill_j = sj;
    s.spill_count = g->d_sctrl + 1;
    s.error = g->d_ctrl + 3;
    if (!ok(imin::launch_decrease_small(s, small_grid(g->num_cus, g->small_launch), st)))
        return IMIN_EDEVICE;
    LargeTarget t{g->d_thr4, s_set, (int32_t)nseeds, reinterpret_cast<unsigned long long *>(d_counts),
                  g->d_stats, g->d_ctrl, ovf, &main_ws, &big_ws};
    rc = launch_large_on(g, t, theta, seed, sj, g->d_sctrl + 1, false);
    if (rc) return rc;

    // Leave the graph's thresholds as created.
    if (!ok(imin::launch_mask_list(thr, orig, g->d_in_ptr, g->d_in_edge, s_set, (int32_t)nseeds,
                                   1, st)))
        return IMIN_EDEVICE;
    if (blocked) {
        hipLaunchKernelGGL(mask_marked_kernel, dim3(grid_of(n)), dim3(kBlock), 0, st, thr, orig,
                           g->d_in_ptr, g->d_in_edge, marks, (int32_t)n, 1);
        if (!ok(hipGetLastError())) return IMIN_EDEVICE;
    }
    unsigned long long sts[kStats];
    uint32_t ctrl[4];
    if (!ok(hipMemcpyAsync(sts, g->d_stats, sizeof(sts), hipMemcpyDeviceToHost, st)) ||
        !ok(hipMemcpyAsync(ctrl, g->d_ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, st)) ||
        !ok(hipEventRecord(g->ev1, st)) || !ok(hipEventSynchronize(g->ev1)))
        return IMIN_EDEVICE;
    g->mask_known = true;
    if (ctrl[3] != 0) return IMIN_EDEVICE;
    if (stats) {
        float ms = 0.0f;
        if (!ok(hipEventElapsedTime(&ms, g->ev0, g->ev1))) return IMIN_EDEVICE;
        stats->samples = sts[0];
        stats->reached = sts[1];
        stats->edges_scanned = sts[2];
        stats->live_edges = sts[3];
        stats->spilled = sts[4];
        stats->wave_samples = sts[5];
        stats->pack_samples = sts[6];
        stats->device_ms = ms;
        stats->kernel_ms = ms;
    }
    return IMIN_OK;
}

}  // extern "C"
