/*
 * imin.h -- C ABI of libimin: GPU estimation of the expected-spread decrease of every
 * candidate blocker from live-edge samples, and the greedy blocker selection built on it,
 * for influence minimisation under the independent cascade model (arXiv 2302.13529).
 *
 * Problem (Section III-B, "Problem Statement"): given a directed graph G = (V, E) with a
 * propagation probability p(u,v) on every edge, a seed set S and a budget b, find a blocker
 * set B, a subset of V \ S with |B| <= b, that minimises the expected spread
 * E(S, G[V \ B]). A blocked vertex never becomes active (Definition 2).
 *
 * Conventions shared by every call:
 *   - Vertices are 0..n-1. Edges are given in CSR form: the out-edges of u are
 *     col[row_ptr[u] .. row_ptr[u+1]-1]; the edge id of an edge is its CSR position.
 *   - Multiple seeds act as one merged source (Section V, "From Multiple Seeds to One
 *     Seed"): a virtual root whose edge to v is live iff at least one seed->v edge is live.
 *     Duplicate seeds are treated as a set. Edges into seeds are irrelevant.
 *   - Live-edge sampling (Definition 4): in sample j of a call whose Philox key is k,
 *     edge e is live iff  (W >> 8) < ceil(p_e * 2^24)  (p_e >= 1: always live), where
 *     W = word (e & 3) of Philox4x32-10 applied to counter (e >> 2, j, 0, 0) with key
 *     (low 32 bits of k, high 32 bits of k) (Salmon et al., SC'11). This is exactly the
 *     float test U < p_e with U = (W >> 8) * 2^-24, so results are a pure function of
 *     (graph, S, blocked set, theta, k) and independent of launch configuration.
 *   - Counts are exact integers. counts[u] = D[u] = sum over samples j < theta of c_j[u],
 *     where c_j[u] is the number of vertices of sample j whose every path from the merged
 *     source passes through u; by Theorem 6 this is the size of u's subtree in the
 *     dominator tree of the sample. The estimated decrease of Algorithm 2 is
 *     Delta[u] = D[u] / theta (Theorem 4); D is returned undivided so ties are exact.
 *   - Every call is synchronous. The caller owns every host array; the library copies its
 *     inputs and keeps no caller pointer after returning. Outputs are written only when the
 *     call returns IMIN_OK; on any error they are left untouched.
 */
#ifndef IMIN_H
#define IMIN_H

#include <stdint.h>

#if defined(__GNUC__)
#define IMIN_API __attribute__((visibility("default")))
#else
#define IMIN_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    IMIN_OK = 0,
    IMIN_EINVAL = -1,  /* an argument violates the contract stated at the call */
    IMIN_ENOMEM = -2,  /* host or device memory could not be allocated */
    IMIN_EDEVICE = -3, /* no usable GPU, or a HIP call failed */
    IMIN_ERANGE = -4   /* a size exceeds what the library supports (e.g. theta > 2^31) */
};

/* Propagation models for imin_graph_create_model. */
enum {
    IMIN_IC = 0, /* independent cascade (Section III-A) */
    IMIN_LT = 1  /* linear threshold, the triggering-model extension (Section V-E) */
};

/* Greedy drivers for imin_greedy. */
enum {
    IMIN_AG = 0, /* AdvancedGreedy, Algorithm 3 */
    IMIN_GR = 1  /* GreedyReplace, Algorithm 4 */
};

/* Opaque handle: the device-resident graph and its per-slot scratch. The calls take it
 * non-const: they write device state it owns (the working thresholds that mask seeds and
 * blockers, the counters, the slots' maps), which is also why calls on one handle must not
 * overlap. The graph itself never changes: each call works from the thresholds as created,
 * restoring whatever an earlier call left masked before it masks its own seeds and
 * blockers. */
typedef struct imin_graph imin_graph;

/* Work counters of a call (summed over every Algorithm 2 call it made). */
typedef struct {
    uint64_t samples;       /* live-edge samples processed (theta per Algorithm 2 call) */
    uint64_t reached;       /* sum over samples of reached non-seed vertices |R_j| */
    uint64_t edges_scanned; /* sum over samples of out-edges of the seeds and of R_j */
    uint64_t live_edges;    /* sum over samples of live edges whose target is neither a
                               seed nor blocked, leaving a seed or a vertex of R_j */
    uint64_t spilled;       /* samples re-run in large-capacity scratch after overflow */
    double device_ms;       /* GPU time of the whole call, measured with HIP events */
    double kernel_ms;       /* GPU time of the sampling/dominator kernel launches alone,
                               summed over the call (HIP events around each launch) */
    uint64_t wave_samples;  /* samples finished by a wavefront-level kernel (one sample per
                               wave, or several per wave); the rest ran one workgroup per
                               sample */
    uint64_t pack_samples;  /* of those, samples finished by the kernel that runs several
                               samples per wavefront (batched calls and the server under
                               the independent cascade model) */
} imin_stats;

/*
 * imin_graph_create -- validate a graph and make it resident on the current HIP device.
 *   n        number of vertices, 1 <= n < 2^31 - 1 (IMIN_ERANGE for n = 2^31 - 1, whose
 *            row_ptr would have 2^31 entries).
 *   m        number of edges, m >= 0; must equal row_ptr[n].
 *   row_ptr  host int32[n+1], row_ptr[0] = 0, non-decreasing.
 *   col      host int32[m], every entry in [0, n). May be NULL when m = 0.
 *   prob     host float[m], the propagation probability p(u,v) of each edge (Section III-A),
 *            each in [0, 1]; NaN is rejected. Self-loops and repeated edges are allowed
 *            (each edge is an independent coin; self-loops never matter).
 *   out      receives the handle; release it with imin_graph_destroy.
 * The probabilities are turned into 24-bit thresholds ceil(p * 2^24) on the host; the
 * device never does floating-point arithmetic on them.
 * Errors: IMIN_EINVAL for any violation above (out is then untouched), IMIN_ERANGE for
 * n = 2^31 - 1, IMIN_ENOMEM, IMIN_EDEVICE.
 */
IMIN_API int imin_graph_create(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                      const float *prob, imin_graph **out);

/*
 * imin_graph_create_model -- as imin_graph_create, under a chosen propagation model.
 *   IMIN_IC  prob[e] is the propagation probability of edge e (imin_graph_create).
 *   IMIN_LT  prob[e] is the weight w(v,u) of edge e = (v,u); the weights of u's in-edges
 *            must sum to at most 1 (up to 1e-5 of rounding; IMIN_EINVAL otherwise). In a
 *            sampled graph u keeps at most one in-edge, each with probability its weight
 *            (u's triggering set, Section V-E): with its in-edges e_1 < e_2 < ... (by edge
 *            id) and bound_k = min(2^24, ceil(2^24 * (w_1 + ... + w_k))) from fp64 running
 *            sums, u keeps e_k in sample j iff bound_{k-1} <= R < bound_k, where R = word
 *            (u & 3) of Philox4x32-10 at counter (u >> 2, j, 1, 0) and the call's key,
 *            shifted right by 8. Every call and greedy driver then works as under IC.
 */
IMIN_API int imin_graph_create_model(int32_t n, int32_t m, const int32_t *row_ptr,
                                     const int32_t *col, const float *prob, int model,
                                     imin_graph **out);

/* Release a handle and all device memory it owns (the graph of imin_graph_create, its
 * workgroup scratch, and the scratch of the batches and servers it leads). No passage of the
 * paper defines this: it is the resource side of the graph residency the calls below rely
 * on. NULL is ignored. */
IMIN_API void imin_graph_destroy(imin_graph *g);

/*
 * imin_decrease -- Algorithm 2 (DecreaseESComputation) on G[V \ B] with exact integer sums.
 *   S, nS    host int32[nS], the seed set; nS >= 1, each seed in [0, n).
 *   blocked  host uint8[n] with 1 for every vertex of B (0 otherwise), or NULL for B empty.
 *            A seed may not be blocked (B is a subset of V \ S, Definition 2).
 *   theta    number of live-edge samples, 1 <= theta <= 2^31 (IMIN_ERANGE above).
 *   seed     the Philox key k of this call.
 *   counts   host uint64[n], receives D[u]; 0 for seeds, blocked and never-reached vertices.
 *   stats    optional (may be NULL), receives the work counters.
 * Errors: IMIN_EINVAL (bad seed, seed blocked, theta = 0, NULL g/S/counts), IMIN_ERANGE
 * (theta > 2^31), IMIN_ENOMEM, IMIN_EDEVICE.
 */
IMIN_API int imin_decrease(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                  uint32_t theta, uint64_t seed, uint64_t *counts, imin_stats *stats);

/*
 * imin_spread -- Monte-Carlo estimate of the expected spread E(S, G[V \ B]) (Definition 1,
 * seeds counted) from theta live-edge samples: by Lemma 1 the number of vertices a sample
 * reaches from S is an unbiased estimate. The samples are those of imin_decrease with the
 * same arguments (same coins), with the dominator work left out.
 *   spread   receives |S| + (sum over samples of reached non-seed vertices) / theta, where
 *            |S| counts distinct seeds; stats->reached holds that exact sum.
 * Other arguments and errors as for imin_decrease (counts replaced by spread).
 */
IMIN_API int imin_spread(imin_graph *g, const int32_t *S, int32_t nS, const uint8_t *blocked,
                         uint32_t theta, uint64_t seed, double *spread, imin_stats *stats);

/*
 * imin_greedy -- AdvancedGreedy (Algorithm 3) or GreedyReplace (Algorithm 4).
 *   b          budget, b >= 0.
 *   theta      samples per Algorithm 2 call, 1 <= theta <= 2^31 (IMIN_ERANGE above).
 *   seed       call r (r = 0, 1, ...) of Algorithm 2 uses Philox key seed + r (mod 2^64),
 *              so round r is bit-identical to imin_decrease with the blockers chosen before
 *              it and key seed + r.
 *   mode       IMIN_AG or IMIN_GR.
 *   blockers   host int32[b], receives the blocker slots in insertion order.
 *   n_blockers receives the number of blockers written.
 *   stats      optional, summed over all Algorithm 2 calls.
 * Argmax ties go to the smallest vertex id; seeds are never candidates.
 *   AG: min(b, n - |S|) rounds; round r blocks argmax of D over V \ (S u B).
 *   GR: CB = out-neighbours of the seeds that are not seeds; min(|CB|, b) rounds pick the
 *       argmax over the remaining CB; then, for each chosen blocker u in reverse insertion
 *       order (over a snapshot of that order), u is unblocked, D is re-estimated, the argmax
 *       x over V \ (S u B) takes u's slot, and the pass stops at the first x == u.
 * Errors: IMIN_EINVAL (as imin_decrease, b < 0, unknown mode, NULL outputs), IMIN_ERANGE
 * (theta > 2^31), IMIN_ENOMEM, IMIN_EDEVICE.
 */
IMIN_API int imin_greedy(imin_graph *g, const int32_t *S, int32_t nS, int32_t b, uint32_t theta,
                uint64_t seed, int mode, int32_t *blockers, int32_t *n_blockers,
                imin_stats *stats);

/*
 * imin_set_launch -- override the launch shape used for later calls on g (0 keeps the
 * automatic choice for that field). slots: concurrent samples, one workgroup each.
 * extra_cap: per-slot capacity for non-tree live edges; samples that exceed it are re-run
 * in large-capacity scratch. Results never depend on these values; they exist so tests can
 * check that, and to tune. Errors: IMIN_EINVAL for negative values or NULL g, IMIN_ERANGE
 * for slots above IMIN_MAX_SLOTS.
 */
#define IMIN_MAX_SLOTS 4096
IMIN_API int imin_set_launch(imin_graph *g, int32_t slots, int64_t extra_cap);

/*
 * Launch shape of the wavefront-level kernels. Every field 0 means "default"; the values
 * change speed only, never results.
 *   waves_per_cu  waves launched per compute unit (default 20; the kernel is persistent,
 *                 so waves beyond what fits on a unit start as others finish).
 *   quad_limit    a 64-vertex frontier chunk with more 4-edge quads than this is left to
 *                 the workgroup kernel (default 2048). The seed level is exempt when its
 *                 rows fit the kernel's 256-quad seed cache.
 *   pick_div      waves take runs of consecutive samples of about a 1/pick_div share of
 *                 what remains per wave, between 4 and 64 samples (default 4).
 *   graph         imin_greedy_batch only: 1 captures all rounds of the call into one HIP
 *                 graph (kernel nodes only) and launches it once; 0 launches them directly.
 */
typedef struct {
    int32_t waves_per_cu;
    int32_t quad_limit;
    int32_t pick_div;
    int32_t graph;
    int32_t pack_per_cu;  /* batched calls and the server: workgroups per compute unit of the
                             kernel that runs several small samples per wavefront (0: the
                             default, 4; -1: that kernel off, every sample starts in the
                             one-sample-per-wave kernel). With it on, its hand-overs go to
                             the workgroup kernel and the other fields have no effect */
} imin_launch;

/*
 * imin_set_small -- policy of the one-wave-per-sample kernel for later calls on g.
 * Every sample first runs in one wavefront with LDS-resident state; a sample that reaches
 * more than 255 vertices, keeps more than 256 non-tree live edges, or meets a frontier
 * chunk over the quad limit is left, with nothing accumulated, to the one-workgroup-per-
 * sample kernel in the same call.
 *   enable  -1 automatic (the default: on for the first round of every call, and off for
 *           the call's later rounds when fewer than half of the first round's samples
 *           finished in the wave kernel; otherwise the second round is timed with it, the
 *           third runs without it as a timed trial, and later rounds keep whichever of the
 *           two was faster), 0 off, 1 on.
 *   launch  the wave kernel's launch shape (NULL: defaults).
 * Results never depend on these values. Errors: IMIN_EINVAL for NULL g, enable outside
 * [-1, 1], or negative launch values.
 */
IMIN_API int imin_set_small(imin_graph *g, int32_t enable, const imin_launch *launch);

/*
 * One problem of a batched greedy call (imin_greedy_batch); the fields mean what the
 * arguments of imin_greedy mean. Outputs are written only when the whole batch succeeds.
 */
typedef struct {
    imin_graph *g;          /* the instance's graph; distinct across one batch */
    const int32_t *S;       /* host int32[nS] seed set */
    int32_t nS;
    int32_t b;              /* budget, b >= 0 */
    uint32_t theta;         /* samples per round, >= 1 */
    uint64_t seed;          /* round r uses Philox key seed + r */
    int32_t *blockers;      /* out: host int32[b] */
    int32_t *n_blockers;    /* out */
    imin_stats *stats;      /* out, may be NULL; device_ms and kernel_ms are the batch's */
} imin_instance;

/*
 * imin_greedy_batch -- AdvancedGreedy (Algorithm 3) or GreedyReplace (Algorithm 4) on `count`
 * independent problems at once. Round r of every instance that still has rounds left runs
 * in the same launches: the wavefront-level kernels over all their samples (samples that
 * outgrow them go to the workgroup kernel), then one argmax per instance, on the device.
 * Under GreedyReplace an instance's round is a first-phase round or a replacement step, and
 * its replacement pass stops on the device; the call reads back one word per round to end
 * when every pass has stopped. Instance i's result is bit-identical to
 * imin_greedy(inst[i].g, S, nS, b, theta, seed, mode, ...).
 * The batch's device scratch (workgroup slots sized for its largest instance, hand-over
 * lists) stays with inst[0].g after the call and serves the next batch that graph leads;
 * imin_graph_destroy releases it.
 *   mode    IMIN_AG or IMIN_GR, for every instance.
 *   count   >= 1; the total of theta over the batch must not exceed 2^31 (IMIN_ERANGE).
 *   launch  the wavefront-level kernels' launch shape (NULL: defaults); the graphs' own
 *           imin_set_small settings do not apply here.
 * Errors: IMIN_EINVAL (any instance invalid as for imin_greedy, a graph repeated, graphs of
 * different models, NULL inst, negative launch values), IMIN_ERANGE, IMIN_ENOMEM,
 * IMIN_EDEVICE.
 */
IMIN_API int imin_greedy_batch(imin_instance *inst, int32_t count, int mode,
                               const imin_launch *launch);

/*
 * Query server: AdvancedGreedy or GreedyReplace for a stream of queries against one resident
 * graph, with continuous batching (see imin_server_step). A query's blockers and counters
 * are those of imin_greedy(g, S, nS, b, theta, seed, mode) alone, whatever else runs beside
 * it.
 */
typedef struct imin_server imin_server;

typedef struct {
    uint64_t hbm_budget;  /* device bytes for per-query state (0: a quarter of free memory) */
    int32_t max_active;   /* most queries admitted at once (0: 256) */
    uint32_t max_theta;   /* largest theta a query may ask for (0: 65536); max_active *
                             max_theta must not exceed 2^31 (IMIN_ERANGE) */
    imin_launch launch;   /* wavefront-level kernels' launch shape, as for imin_greedy_batch
                             (zeros: defaults; its graph field is not used) */
} imin_server_config;

/*
 * imin_server_create -- a server for graph g (cfg may be NULL for defaults). The server
 * reads g's resident arrays and never changes them; g must outlive the server. Errors:
 * IMIN_EINVAL, IMIN_ERANGE, IMIN_ENOMEM (budget or scratch not allocatable), IMIN_EDEVICE.
 */
IMIN_API int imin_server_create(imin_graph *g, const imin_server_config *cfg, imin_server **out);

/* Release a server and its device memory (pending queries are dropped). NULL is ignored. */
IMIN_API void imin_server_destroy(imin_server *s);

/* Device bytes a query with nS distinct seeds and budget b holds while admitted. */
IMIN_API int imin_server_query_bytes(const imin_server *s, int32_t nS, int32_t b,
                                     uint64_t *bytes);

/*
 * imin_server_submit -- queue a query (arguments as for imin_greedy with IMIN_AG) and
 * receive its ticket. Nothing runs until imin_server_step. Errors: IMIN_EINVAL as for
 * imin_greedy; IMIN_ERANGE when theta > max_theta or the query's state can never fit the
 * budget.
 */
IMIN_API int imin_server_submit(imin_server *s, const int32_t *S, int32_t nS, int32_t b,
                                uint32_t theta, uint64_t seed, uint64_t *ticket);

/*
 * imin_server_submit_mode -- as imin_server_submit, with the greedy driver: IMIN_AG
 * (Algorithm 3) or IMIN_GR (Algorithm 4; its replacement pass stops on the device, and the
 * query retires at the step where it stops). Errors: as imin_server_submit, and IMIN_EINVAL
 * for an unknown mode.
 */
IMIN_API int imin_server_submit_mode(imin_server *s, const int32_t *S, int32_t nS, int32_t b,
                                     uint32_t theta, uint64_t seed, int mode, uint64_t *ticket);

/*
 * imin_server_step -- one scheduling step: admit queued queries in arrival order while
 * their state fits the budget and fewer than max_active are admitted (a query that does
 * not fit waits, and so do the ones behind it); run one greedy round of every admitted
 * query in shared launches; retire the queries whose rounds are done (GreedyReplace: or
 * whose replacement pass stopped in this step). Returns when the
 * step's GPU work has finished. n_active / n_queued (nullable) receive the counts after
 * the step.
 */
IMIN_API int imin_server_step(imin_server *s, int32_t *n_active, int32_t *n_queued);

/* Pop up to cap tickets of queries finished since the last call, oldest first. */
IMIN_API int imin_server_completed(imin_server *s, uint64_t *tickets, int32_t cap,
                                   int32_t *count);

/*
 * imin_server_result -- take a finished query's blockers (capacity cap) and counters
 * (device_ms and kernel_ms are 0). Returns IMIN_OK once, then forgets the ticket; 1 while
 * the query is queued or running; IMIN_EINVAL for an unknown ticket; IMIN_ERANGE when cap is
 * too small (the result stays available).
 */
IMIN_API int imin_server_result(imin_server *s, uint64_t ticket, int32_t *blockers, int32_t cap,
                                int32_t *n_blockers, imin_stats *stats);

/*
 * imin_decrease_noalloc -- imin_decrease for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * It computes the same counts and work counters as imin_decrease with the same arguments,
 * and calls no hipMalloc, hipFree or other allocating routine: every scratch buffer of the
 * call (seed staging, blocked marks, hand-over and overflow lists, the per-slot maps,
 * records and extra-edge lists of the workgroup kernel, its large-capacity spill slots) is
 * carved from one static device array of IMIN_NOALLOC_SCRATCH_BYTES per GPU, which each GPU
 * the library runs on holds until the process ends.
 *   g, S, nS, blocked, theta, seed   as for imin_decrease.
 *   d_counts  DEVICE pointer to uint64[n] on g's device, owned by the caller; receives D
 *             (written only by the kernels; its contents are undefined if the call fails).
 *   stats     optional host struct, as for imin_decrease (device_ms and kernel_ms are both
 *             the whole call).
 * Limits: the graph's scratch must fit the array -- per workgroup slot about 30 * (n + 1)
 * bytes (38 * (n + 1) under IC, whose slots also keep each reached vertex's row range),
 * plus two large-capacity slots of about that much plus 8 * m bytes when a slot's
 * extra-edge list cannot hold m edges, plus 8 * theta + 8 * nS bytes of lists and n / 8 + n
 * bytes of seed bits and blocked marks -- else IMIN_ERANGE (for example a 2^17-vertex,
 * 10^6-edge graph fits; a 2^22-vertex one does not). Fewer slots than imin_decrease uses
 * may fit, which costs speed, never results.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one GPU race;
 * the call clears what must start at zero and leaves the graph's thresholds as created.
 * Errors: IMIN_EINVAL (as imin_decrease, or d_counts NULL), IMIN_ERANGE, IMIN_EDEVICE.
 */
#define IMIN_NOALLOC_SCRATCH_BYTES (256u << 20)
IMIN_API int imin_decrease_noalloc(imin_graph *g, const int32_t *S, int32_t nS,
                                   const uint8_t *blocked, uint32_t theta, uint64_t seed,
                                   uint64_t *d_counts, imin_stats *stats);

/* Human-readable text of a status code (static storage). An interface convenience; no
 * passage of the paper defines it. */
IMIN_API const char *imin_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* IMIN_H */
