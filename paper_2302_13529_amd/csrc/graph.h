// graph.h -- the host-side graph handle of libimin and the helpers its C entry points share
// (api.cpp: single and batched calls; server.cpp: the query server).
#pragma once

#include "imin.h"
#include "imin_internal.h"

#include <vector>

namespace imin {
namespace host {
struct MultiScratch;
}  // namespace host
}  // namespace imin

struct imin_graph {
    int device = 0;
    int32_t n = 0;
    int32_t m = 0;
    int num_cus = 1;
    std::vector<int32_t> row_ptr;  // host copies: out-neighbours of the seeds (GR)
    std::vector<int32_t> col;
    int32_t *d_row_ptr = nullptr;
    uint4 *d_col4 = nullptr;      // edge targets, 4 per quad, padded to a whole quad
    uint4 *d_edge = nullptr;      // independent cascade: one record per edge slot of d_col4,
                                  // (target, target's row start, row end, 0)
    uint4 *d_thr4 = nullptr;      // working live thresholds, same layout: 0 on every edge into
                                  // a vertex of `masked`
    uint4 *d_thr_orig = nullptr;  // the thresholds ceil(p * 2^24) as created
    int model = 0;                // IMIN_IC or IMIN_LT
    uint4 *d_lo4 = nullptr;       // linear-threshold model: interval lower bounds
    uint4 *d_tl = nullptr;        // linear-threshold model: per quad, its targets and then its
                                  // lower bounds (32 bytes, one line)
    int32_t *d_in_ptr = nullptr;  // in-edges of v: d_in_edge[d_in_ptr[v] .. d_in_ptr[v+1])
    int32_t *d_in_edge = nullptr; // edge ids, grouped by target
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t words = 0;                       // 32-bit words of a vertex bitmap
    uint32_t *d_inelig = nullptr;            // seeds and blocked vertices
    uint32_t *d_cand = nullptr;              // GR candidate set CB
    int32_t *d_seeds = nullptr;              // distinct seeds (capacity n)
    unsigned long long *d_D = nullptr;       // n
    unsigned long long *d_stats = nullptr;   // kStats: samples, reached, scanned, live,
                                             // spilled, wave-kernel samples
    uint32_t *d_ctrl = nullptr;              // kCtrlWords: next main, next spill, spill count,
                                             // error (in batched calls: the instance's words)
    uint32_t *d_sctrl = nullptr;             // 2: wave-kernel work counter, samples it left
    uint32_t *d_sj = nullptr;                // samples the wave kernel left to the large one
    uint32_t sj_cap = 0;
    imin::InstanceDesc *d_inst = nullptr;    // this graph as the one instance of a wave launch
    imin::InstanceDesc h_inst{};
    int small_mode = -1;                     // wave kernel: -1 automatic, 0 off, 1 on
    bool small_auto_off = false;             // automatic mode: this call's first round found
                                             // most samples too large
    bool auto_pending = false;               // wave kernel on: this call's first round not yet judged
    int probe = 0;                           // automatic mode, per call: 1 = time the next
                                             // round (wave kernel on), 2 = the next round is a
                                             // timed trial without it, 3 = compare; 0 = none
    size_t probe_kev[2] = {0, 0};            // kev index of the timed rounds (with, without)
    imin_launch small_launch{};              // 0 fields: defaults
    uint32_t *d_ovf = nullptr;
    uint32_t ovf_cap = 0;
    unsigned long long *d_part_d = nullptr;
    int32_t *d_part_i = nullptr;
    int32_t parts = 4096;
    int32_t *d_B = nullptr;
    int32_t B_cap = 0;
    int32_t *d_x = nullptr;
    imin::Workspace main_ws, big_ws;
    std::vector<int32_t> masked;       // vertices whose in-edges have threshold 0 in d_thr4
    std::vector<int32_t> mask_prev;    // the previous call's list, kept while copies run
    bool mask_known = true;            // false while a call runs, and after one that failed
    int32_t *d_list = nullptr;         // 2n: device copies of the two lists above
    std::vector<hipEvent_t> kev;  // pairs around each decrease launch of the current call
    size_t kev_used = 0;
    imin::host::MultiScratch *batch_ms = nullptr;  // scratch of the batches this graph leads
                                                   // (first instance), kept for the next one
    int32_t force_slots = 0;
    int64_t force_xcap = 0;
};

namespace imin {
namespace host {

constexpr int kStats = 7;  // samples, reached, scanned, live, spilled, wave-level kernel
                           // samples, packed-kernel samples
// The per-launch work counter is 32-bit and every workgroup takes one index past the end.
constexpr uint32_t kMaxTheta = 1u << 31;

inline bool ok(hipError_t e) { return e == hipSuccess; }

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_ws(Workspace &ws);
// Scratch of `slots` workgroup-kernel slots with maps of n entries (kept when the shape is
// unchanged); cleared on `stream`. rng: with the per-local-vertex row ranges that the
// many-instance kernel keeps.
int alloc_ws(Workspace &ws, int64_t n, int32_t slots, int64_t lcap, int64_t xcap,
             hipStream_t stream, bool rng);
// Validated seed set: distinct seeds ascending, and the seed bitmap.
int seed_setup(imin_graph *g, const int32_t *S, int32_t nS, std::vector<int32_t> &seeds,
               std::vector<uint32_t> &inelig);
int small_grid(int num_cus, const imin_launch &l);
void small_shape(SmallArgs &s, const imin_launch &l);
bool launch_ok(const imin_launch *l);

// Where a workgroup-kernel launch reads its call state and accumulates: the graph's own
// buffers for single calls, a query's for the server.
struct LargeTarget {
    const uint4 *thr4;
    const int32_t *seeds;
    int32_t nseeds;
    unsigned long long *D;
    unsigned long long *stats;
    uint32_t *ctrl;      // 4 words: next main, next spill, spill count, error
    uint32_t *ovf;       // capacity >= theta
    Workspace *main_ws;  // slots > 0
    Workspace *big_ws;   // slots == 0 when no sample can overflow main_ws
};
// The workgroup kernel over samples 0..theta-1, or over the device list `list` of *count
// samples, then the large-scratch launch for the samples that overflowed.
int launch_large_on(imin_graph *g, const LargeTarget &t, uint32_t theta, uint64_t key,
                    const uint32_t *list, const uint32_t *count, bool reach_only);

// Device scratch of rounds over many instances at once (batched calls, the server): the
// wave kernel's hand-over list, the workgroup kernel's slots (maps sized for the largest
// instance) and its own overflow list, and the control words of one round.
constexpr int kMultiCtrl = 10;

struct MultiScratch {
    int64_t n = 0, m = 0;      // largest instance it serves
    uint32_t cap = 0;          // samples of the largest round
    Workspace main_ws, big_ws;
    uint32_t *ctrl = nullptr;  // kMultiCtrl: wave next, wave hand-overs, wave error, main
                               // next, big next, overflow count, workgroup error, packed
                               // hand-overs, packed next, instances done this call
    uint32_t *pi = nullptr, *pj = nullptr;  // packed kernel's hand-over list: instance, sample
    uint32_t *si = nullptr, *sj = nullptr;  // wave kernel's hand-over list: instance, sample
    uint32_t *oi = nullptr, *oj = nullptr;  // overflow list: instance, sample
    int32_t inst_cap = 0;                   // instances of the largest round
    unsigned long long *part_d = nullptr;   // inst_cap * kArgParts partial argmax results
    int32_t *part_i = nullptr;
    // Batched calls: the instance table and call-state staging, kept across calls (grown on
    // demand), and the HIP graph of the last captured call with the launch structure it was
    // captured for (replayed while a call has the same structure).
    InstanceDesc *table = nullptr;
    size_t table_cap = 0;
    BatchStage *stages = nullptr;
    size_t stages_cap = 0;
    int32_t *stage = nullptr;
    size_t stage_cap = 0;
    int32_t *rounds = nullptr;
    size_t rounds_cap = 0;
    int32_t *out = nullptr;
    size_t out_cap = 0;
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> exec_key;
};
int multi_alloc(MultiScratch &ms, int num_cus, int64_t max_n, int64_t max_m, uint32_t cap,
                int32_t max_inst, hipStream_t stream);
void multi_free(MultiScratch &ms);
// One round of every instance of the device table inst[0..ninst) (sample indices
// [0, total), keys seed + round, greedy round step + round): for GreedyReplace instances in
// their replacement pass (gr) the unblocking of that round's slot, then the wavefront-level
// kernels, the workgroup kernels for the samples they hand over, then (select) each
// instance's greedy choice, applied (launch_batch_argmax; instances that end their run add
// one to ms.ctrl[9]). Nothing waits for the host. D is cleared first.
int multi_round(MultiScratch &ms, const InstanceDesc *inst, int32_t ninst, uint32_t total,
                uint32_t round, const imin_launch &shape, int num_cus, bool select, bool gr,
                bool lt, hipStream_t stream);
// GreedyReplace's first-phase candidates CB = out-neighbours of the seeds that are not
// seeds, as a bitmap over g's vertices; returns |CB|.
int32_t gr_candidates(const imin_graph *g, const std::vector<int32_t> &seeds,
                      const std::vector<uint32_t> &inelig, std::vector<uint32_t> &cand);
// The error words of the last rounds (0 when every sample was counted).
int multi_errors(MultiScratch &ms, uint32_t *wave_err, uint32_t *wg_err, hipStream_t stream);

}  // namespace host
}  // namespace imin
