// imin_internal.h -- shapes shared by the host API and the HIP kernels of libimin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imin {

// Threads per workgroup of the workgroup-per-sample kernel (one workgroup works on one sample
// at a time): single calls, whose samples may be huge, and many-instance launches (batched
// calls, the server), whose handed-over samples are mostly of moderate size and gain more
// from having more of them in flight.
constexpr int kBlock = 1024;
constexpr int kMultiBlock = 256;
// Workgroup slots per compute unit: as many as its 32 wave slots hold.
constexpr int kSlotsPerCu = 2048 / kBlock;
constexpr int kMultiSlotsPerCu = 2048 / kMultiBlock;

// Seeds and blocked vertices: every edge into such a vertex has live threshold 0 in the
// graph's working threshold array while a call runs, so it is never live, which is exactly
// the rule that a live edge never activates a seed again or a blocked vertex (Definition 2;
// each edge's coin is independent of the others). The kernels therefore never test it.

// Per slot and vertex, one 64-bit map entry. Its high word is (epoch << lbits) | (lid + 1),
// the epoch of the sample that last reached the vertex above its local id in that sample;
// its low word counts the launch's samples in this slot that reached the vertex. A sample
// with epoch t claims a vertex by a 64-bit atomic max with (t << lbits) << 32: the entry was
// below that value exactly when the vertex was not yet reached in this sample, and the
// atomic returns the old count. The claimer then stores its local id and the count plus one
// in one store (a later max by the same sample leaves the larger value in place); a lid
// field of 0 means "claimed, local id not yet written". Counting each reached vertex's 1 in
// its decrease count this way costs no memory access beyond the claim, and only subtree
// sizes above 1 go to the device-wide counters (single-problem launches; many-instance
// launches keep the count at 0 and add every size to D). When a slot's epoch reaches the
// largest value the high word holds, the slot clears its high words and starts again from
// epoch 1.

// Per slot and local vertex (local id 0 is the merged seed): the vertex id, the parent in
// the BFS spanning tree, the tentative immediate dominator and the subtree size. One
// 16-byte record, written once when the vertex is reached.
struct LocalVtx {
    int32_t glob;
    int32_t par0;
    int32_t tdom;
    int32_t csz;
};

// Scratch of `slots` concurrent samples. Arrays are slot-major: slot s owns
// [s * n, (s + 1) * n) of `map`, [s * lcap, (s + 1) * lcap) of `loc`, and so on.
struct Workspace {
    int32_t slots = 0;
    int64_t n = 0;             // map entries per slot (vertex ids below n)
    int64_t lcap = 0;          // local vertices per sample (root included)
    int64_t xcap = 0;          // non-tree live edges per sample
    unsigned long long *map = nullptr;  // slots * n
    int32_t lbits = 0;         // bits of the local-id field: lcap < 2^lbits, lbits <= 31
    LocalVtx *loc = nullptr;   // slots * lcap
    int32_t *lvl = nullptr;    // slots * (lcap + 1): first local id of each BFS level
    int2 *extra = nullptr;     // slots * xcap: (source local id, target vertex -> local id)
    int2 *rng = nullptr;       // slots * lcap, except for linear-threshold single calls: the
                               // row range (row_ptr pair) of each local vertex, known when it
                               // is claimed
    uint32_t *epoch = nullptr; // slots: epoch of the slot's last sample
    uint32_t *dirty = nullptr; // slots: 1 when the slot's last counting launch left reach
                               // counts in its map (launch_flush_counts reads only those)
    size_t bytes = 0;
};

struct InstanceDesc;

// Everything one launch of the decrease kernel reads or writes.
struct DecreaseArgs {
    const int32_t *row_ptr;  // n + 1
    const uint4 *col4;       // ceil(m / 4) quads of edge targets (4 edges = 16 bytes)
    const uint4 *edge;       // single calls under IC: 4 * ceil(m / 4) records (target,
                             // target's row start, row end, 0), so that a live edge's one
                             // line also gives the row the next level expands
    const uint4 *thr4;       // ceil(m / 4) quads of live thresholds ceil(p * 2^24), 0 for
                             // edges into seeds and blocked vertices
    const uint4 *lo4;        // linear-threshold model: interval lower bounds (thr4 = upper)
    const uint4 *tl;         // linear-threshold model: 2 * ceil(m / 4) quads, quad q's targets
                             // at 2q and its lower bounds at 2q + 1
    int32_t lt;              // 1: linear-threshold model, 0: independent cascade
    const int32_t *seeds;    // distinct seeds
    int32_t nseeds;
    int32_t n;
    uint32_t key_lo, key_hi; // Philox key of the call
    uint32_t theta;          // samples 0..theta-1 when sample_list is null
    const uint32_t *sample_list;   // else: samples sample_list[0..*sample_count)
    const uint32_t *sample_count;
    uint32_t *next;          // work counter of this launch
    unsigned long long *D;   // n decrease counters
    unsigned long long *stats; // samples, reached, edges scanned, live edges
    uint32_t *ovf_list;      // samples whose scratch overflowed (when spill_ok)
    uint32_t *ovf_count;
    uint32_t *error;         // set when a sample overflows with spill_ok == 0
    int32_t spill_ok;
    int32_t reach_only;      // count reached vertices only (spread estimates)
    int32_t count_reach;     // a slot may add each reached vertex's 1 into its map entry
                             // instead of D (the caller folds them into D with
                             // launch_flush_counts); each slot decides after its first
                             // sample and records the choice in ws.dirty
    Workspace ws;            // slot maps of `n` entries
    // Many-instance launches (inst non-null): sample idx is sample sample_list[idx] of
    // instance inst[sample_inst[idx]] with key seed + round; overflowing samples are
    // listed with their instance in ovf_inst. Every instance's n must be <= n.
    const InstanceDesc *inst;
    const uint32_t *sample_inst;
    uint32_t *ovf_inst;
    uint32_t round;
};

// decrease.hip
hipError_t launch_decrease(const DecreaseArgs &a, hipStream_t stream);
// D[v] += the reach counts of v in the first `slots` slots of ws, which are cleared.
hipError_t launch_flush_counts(const Workspace &ws, int32_t slots, unsigned long long *D,
                               hipStream_t stream);

// Wave-per-sample kernel (small.hip): per-sample capacity in local vertices (root
// included) and in non-tree live edges, and waves per workgroup.
constexpr int kSmallV = 256;
constexpr int kSmallX = 256;
constexpr int kSmallWaves = 4;

// One problem instance of a wave-kernel launch: a resident graph, its seed set and
// seed/blocked bitmap, and its counters. Samples [sample_base, sample_base + theta) of the
// launch belong to it; sample j of the instance uses Philox key seed + round.
struct InstanceDesc {
    const int32_t *row_ptr;
    const uint4 *col4;
    const uint4 *edge;        // independent cascade: per-edge records (target, target's row
                              // start, row end, 0), as DecreaseArgs::edge
    uint4 *thr4;              // working thresholds (the batched argmax masks its winners)
    const uint4 *lo4;         // linear-threshold model: interval lower bounds
    const uint4 *tl;          // linear-threshold model: targets and lower bounds, as
                              // DecreaseArgs::tl
    const int32_t *in_ptr;    // in-edges of v: in_edge[in_ptr[v] .. in_ptr[v+1])
    const int32_t *in_edge;   // edge ids
    uint32_t *inelig;         // bit v set: v is a seed or blocked (the argmax adds winners)
    const int32_t *seeds;
    unsigned long long *D;    // n decrease counters
    unsigned long long *stats; // samples, reached, edges scanned, live edges, -, wave-level
                               // kernel samples, packed-kernel samples
    int32_t *B;               // blocker slots (batched greedy)
    int32_t *x;               // the last round's winner (batched greedy)
    const uint4 *thr_orig;    // thresholds as created (batched set-up restores from them)
    uint32_t *ctrl;           // kCtrlWords control words: the graph's workgroup-kernel
                              // counters in single calls; in many-instance launches see
                              // kCtrlSkipWave .. kCtrlPackHanded
    uint32_t *cand;           // GreedyReplace: its first phase's candidate set CB (bit v set)
    int32_t gr_k;             // GreedyReplace: rounds of its first phase, k = min(|CB|, b);
                              // -1: AdvancedGreedy
    int32_t step;             // the instance's round is step + the launch's round (the call
                              // index of its greedy run; blocker slot of AdvancedGreedy)
    int32_t nseeds;
    int32_t n;
    int32_t nquads;           // quads of thr4
    uint32_t seed_lo, seed_hi;
    uint32_t theta;
    uint32_t sample_base;
};

// Control words of an instance in many-instance launches (InstanceDesc::ctrl).
constexpr int kCtrlWords = 8;
constexpr int kCtrlSkipWave = 0;    // 1: the wave kernel lists the instance's samples onward
constexpr int kCtrlWaveHanded = 1;  // samples the wave kernel handed over this round
constexpr int kCtrlError = 3;       // nonzero: a sample was lost (never expected)
constexpr int kCtrlSkipPack = 4;    // 1: the packed kernel lists the instance's samples onward
constexpr int kCtrlPackHanded = 5;  // samples the packed kernel handed over this round
constexpr int kCtrlDone = 6;        // 1: the instance's greedy run has ended (GreedyReplace's
                                    // replacement pass stopped); its samples are skipped

struct SmallArgs {
    const InstanceDesc *inst; // ascending sample_base
    int32_t ninst;
    uint32_t total;           // samples of the launch: sum of the instances' theta
    uint32_t round;           // added to every instance's seed to form the key
    int32_t quad_limit;       // a frontier chunk with more edge quads goes to the large kernel
    int32_t pick_div;         // runs of samples: about remaining / (pick_div * waves)
    int32_t lt;               // every instance uses the linear-threshold model
    int32_t reach_only;       // count reached vertices only (spread estimates)
    uint32_t *next;           // work counter
    uint32_t *spill_inst;     // samples left to the large kernel: instance, sample index
    uint32_t *spill_j;
    uint32_t *spill_count;
    uint32_t *error;          // bit 2: dominator iteration did not settle (never expected)
};

// small.hip
hipError_t launch_decrease_small(const SmallArgs &a, int grid, hipStream_t stream);

// Packed wave kernel (pack.hip): kPackG samples of one instance share a wavefront, each with
// capacity kPackV local vertices (root included) and kPackX non-tree live edges, its reached
// set kept in an LDS hash table of kPackH slots. Independent cascade only.
constexpr int kPackG = 4;
constexpr int kPackV = 64;
constexpr int kPackX = 64;
constexpr int kPackH = 128;
constexpr int kPackWaves = 4;

struct PackArgs {
    const InstanceDesc *inst; // ascending sample_base
    int32_t ninst;
    uint32_t total;           // samples of the launch: sum of the instances' theta
    uint32_t round;           // added to every instance's seed to form the key
    int32_t quad_limit;       // a frontier vertex with more edge quads is handed over
    int32_t pick_div;         // runs of samples: about remaining / (pick_div * waves)
    uint32_t *next;           // work counter
    uint32_t *out_inst;       // samples handed to the workgroup kernel: instance, sample
    uint32_t *out_j;
    uint32_t *out_count;
    uint32_t *error;          // bit 2: dominator iteration did not settle (never expected)
};

hipError_t launch_decrease_pack(const PackArgs &a, int grid, hipStream_t stream);

// select.hip
hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long value,
                           hipStream_t stream);
hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t stream);
// Argmax of D over candidates (mode 0: bit of `bits` clear; mode 1: bit of `bits` set),
// ties to the smallest id. Then: set the winner's bit in `inelig`, clear it in `cand`
// (if non-null), store it in B[slot] and *out_x, and give its in-edges threshold 0 in `thr`.
// *out_x = -1 when there is no candidate.
hipError_t launch_argmax_apply(const unsigned long long *D, const uint32_t *bits, int mode,
                               int32_t n, unsigned long long *part_d, int32_t *part_i,
                               int32_t parts, uint32_t *inelig, uint32_t *cand, int32_t *B,
                               int32_t slot, int32_t *out_x, uint32_t *thr,
                               const int32_t *in_ptr, const int32_t *in_edge,
                               hipStream_t stream);
hipError_t launch_set_bit(uint32_t *bits, int32_t v, int value, hipStream_t stream);
// Thresholds of the in-edges of the vertices list[0..count) (device list), or of the one
// vertex v (host value; or the device-resident id at v_dev when v_dev is non-null, ignored
// when negative): set to 0 (restore == 0) or copied back from thr_orig (restore != 0).
hipError_t launch_mask_list(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                            const int32_t *in_edge, const int32_t *list, int32_t count,
                            int restore, hipStream_t stream);
hipError_t launch_mask_vertex(uint32_t *thr, const uint32_t *thr_orig, const int32_t *in_ptr,
                              const int32_t *in_edge, int32_t v, const int32_t *v_dev,
                              int restore, hipStream_t stream);
// Batched greedy over instances inst[0..ninst): zero every instance's D; and per instance,
// the AdvancedGreedy selection (argmax of D over vertices whose inelig bit is clear, ties to
// the smallest id), applied as launch_argmax_apply does, with the winner in B[slot] and *x
// and its in-edges masked in the instance's thresholds.
hipError_t launch_batch_zero(const InstanceDesc *inst, int32_t ninst, hipStream_t stream);

// Per-instance call state of a batched call, staged in one device buffer `stage`:
// seeds at [seeds, seeds + nseeds), the seed/blocked bitmap at [bits, bits + words), the
// vertices the previous call left masked at [prev, prev + nprev) (nprev < 0: restore every
// threshold), and the vertices to mask now at [now, now + nnow).
struct BatchStage {
    int64_t seeds, bits, prev, now;
    int32_t words, nprev, nnow, pad;
    int64_t cand;  // GreedyReplace: CB bitmap at [cand, cand + words); -1: none
};
// One workgroup per instance: copy seeds and bitmap into place, clear the counters and
// control words, restore the previous masks, then mask the new ones.
hipError_t launch_batch_setup(const InstanceDesc *inst, const BatchStage *st,
                              const int32_t *stage, int32_t ninst, hipStream_t stream);
// One workgroup per instance: B[0..rounds[i]), the 6 counters and control word 3 of
// instance i into out + i * stride (int32 words; counters as pairs of words).
hipError_t launch_batch_gather(const InstanceDesc *inst, const int32_t *rounds, int32_t *out,
                               int32_t stride, int32_t ninst, hipStream_t stream);
// The greedy choice of every instance in its round (step + round) and its application:
// kArgParts workgroups per instance scan a share of its D each and leave their best
// (D, vertex) in part_d/part_i (ninst * kArgParts entries); one workgroup per instance then
// reduces them and applies the winner x (bitmap bit, in-edge masks, *x):
//   AdvancedGreedy (Algorithm 3): argmax over V \ (S u B) into B[step];
//   GreedyReplace (Algorithm 4), first phase (step < k): argmax over the remaining CB into
//     B[step], x leaves CB;
//   GreedyReplace, replacement pass (k <= step < 2k): slot i = 2k - 1 - step, whose blocker
//     u was unblocked before the round's samples (launch_batch_gr_prepare); argmax over
//     V \ (S u B) into B[i]; the instance is done when x == u or i == 0 (*done_count + 1).
// Instances already done are skipped.
constexpr int kArgParts = 16;
// Layout of one instance's record in the batch gather buffer (int32 words): the kGatherStats
// 64-bit counters as pairs of words, the error word, then the blocker slots.
constexpr int kGatherStats = 7;
constexpr int kGatherErr = 2 * kGatherStats;
constexpr int kGatherB = kGatherErr + 1;
hipError_t launch_batch_argmax(const InstanceDesc *inst, int32_t ninst, int32_t round,
                               unsigned long long *part_d, int32_t *part_i, uint32_t *done_count,
                               hipStream_t stream);
// GreedyReplace instances in their replacement pass: unblock the blocker of slot
// 2k - 1 - (step + round) (bitmap bit cleared, in-edge thresholds restored) before the
// round's samples. Other instances are left alone.
hipError_t launch_batch_gr_prepare(const InstanceDesc *inst, int32_t ninst, int32_t round,
                                   hipStream_t stream);
// out[i] = the done word of instance i.
hipError_t launch_batch_done(const InstanceDesc *inst, int32_t ninst, uint32_t *out,
                             hipStream_t stream);

}  // namespace imin
