// server.cpp -- the query server of libimin: AdvancedGreedy or GreedyReplace (Algorithms 3
// and 4 of arXiv 2302.13529) for a stream of (S, b, theta, seed) queries against one
// resident graph, with continuous batching.
//
// Every query owns its state on the device: a copy of the graph's live thresholds (its seeds
// and blockers get threshold 0 on their in-edges, as in a single call), the seed/blocked
// bitmap, its seeds, counters D, work counters and blocker slots. That state is carved out
// of one pool allocated when the server starts; a queued query is admitted, in arrival
// order, as soon as its state fits in the pool and a slot is free. A step runs one greedy
// round of every admitted query in shared launches (the wavefront-level kernels over all
// their samples, the workgroup kernels for the samples they hand over, one argmax per query),
// then retires the queries that have made all their rounds -- or, under GreedyReplace, whose
// replacement pass has stopped (a device-side flag read back with the step). A query's key
// for round r is seed + r, so a query's blockers and counters are those of imin_greedy alone,
// whatever else shares its steps.
#include "graph.h"

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <unordered_set>
#include <vector>

using namespace imin::host;

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kDefaultMaxActive = 256;
constexpr uint32_t kDefaultMaxTheta = 1u << 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device range, with coalescing of free neighbours.
class Pool {
  public:
    bool init(size_t bytes)
    {
        bytes = bytes / kAlign * kAlign;
        if (bytes == 0 || !ok(hipMalloc(&base_, bytes))) {
            (void)hipGetLastError();
            base_ = nullptr;
            return false;
        }
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    ~Pool()
    {
        if (base_) (void)hipFree(base_);
    }
    size_t size() const { return size_; }
    // Offset of a free range of `bytes`, or SIZE_MAX.
    size_t alloc(size_t bytes)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    char *at(size_t off) const { return base_ + off; }

  private:
    char *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Query {
    uint64_t ticket = 0;
    std::vector<int32_t> seeds;
    std::vector<uint32_t> inelig;
    std::vector<uint32_t> cand;  // GreedyReplace: CB
    int32_t b = 0, rounds = 0, round = 0;
    int32_t mode = IMIN_AG;
    int32_t nb = 0;              // blocker slots (GreedyReplace: k)
    uint32_t theta = 0;
    uint64_t seed = 0;
    size_t off = 0, bytes = 0;
    imin::InstanceDesc desc{};  // device pointers into the pool
};

struct Result {
    std::vector<int32_t> B;
    imin_stats stats{};
};

}  // namespace

struct imin_server {
    imin_graph *g = nullptr;
    hipStream_t stream = nullptr;
    imin_server_config cfg{};
    Pool pool;
    MultiScratch ms;
    std::deque<Query> queue;
    std::vector<Query> active;
    std::unordered_map<uint64_t, Result> done;
    std::unordered_set<uint64_t> pending;  // queued or active
    std::vector<uint64_t> completed;
    uint64_t next_ticket = 1;
    // per-step host staging, alive until the step's wait
    std::vector<imin::InstanceDesc> table;
    std::vector<imin::BatchStage> stages;
    std::vector<int32_t> stage, rounds, out;
    // device buffers of the step tables, sized for max_active
    imin::InstanceDesc *d_table = nullptr;
    imin::BatchStage *d_stages = nullptr;
    int32_t *d_stage = nullptr;
    size_t stage_cap = 0;
    int32_t *d_rounds = nullptr;
    int32_t *d_out = nullptr;
    size_t out_cap = 0;
};

namespace {

// Pool bytes of one query: thresholds, bitmap, candidate bitmap, seeds, D, counters, control
// words, blockers.
size_t footprint(const imin_graph *g, int32_t nseeds, int32_t b)
{
    const size_t quads = (size_t)std::max<int64_t>(((int64_t)g->m + 3) / 4, 1);
    return align_up(quads * sizeof(uint4)) + 2 * align_up((size_t)g->words * 4) +
           align_up((size_t)std::max(nseeds, 1) * 4) + align_up((size_t)g->n * 8) +
           align_up(kStats * 8) + align_up(imin::kCtrlWords * 4) + align_up((size_t)std::max(b, 1) * 4) +
           align_up(4);
}

// Device pointers of a query's state at pool offset q.off.
void carve(imin_server *s, Query &q)
{
    imin_graph *g = s->g;
    char *p = s->pool.at(q.off);
    const size_t quads = (size_t)std::max<int64_t>(((int64_t)g->m + 3) / 4, 1);
    imin::InstanceDesc &I = q.desc;
    std::memset(&I, 0, sizeof(I));
    I.thr4 = reinterpret_cast<uint4 *>(p);
    p += align_up(quads * sizeof(uint4));
    I.inelig = reinterpret_cast<uint32_t *>(p);
    p += align_up((size_t)g->words * 4);
    I.cand = reinterpret_cast<uint32_t *>(p);
    p += align_up((size_t)g->words * 4);
    I.seeds = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)std::max<size_t>(q.seeds.size(), 1) * 4);
    I.D = reinterpret_cast<unsigned long long *>(p);
    p += align_up((size_t)g->n * 8);
    I.stats = reinterpret_cast<unsigned long long *>(p);
    p += align_up(kStats * 8);
    I.ctrl = reinterpret_cast<uint32_t *>(p);
    p += align_up(imin::kCtrlWords * 4);
    I.B = reinterpret_cast<int32_t *>(p);
    p += align_up((size_t)std::max(q.b, 1) * 4);
    I.x = reinterpret_cast<int32_t *>(p);
    I.row_ptr = g->d_row_ptr;
    I.col4 = g->d_col4;
    I.edge = g->d_edge;
    I.lo4 = g->d_lo4;
    I.tl = g->d_tl;
    I.in_ptr = g->d_in_ptr;
    I.in_edge = g->d_in_edge;
    I.thr_orig = g->d_thr_orig;
    I.nseeds = (int32_t)q.seeds.size();
    I.n = g->n;
    I.nquads = (int32_t)quads;
    I.theta = q.theta;
    I.gr_k = q.mode == IMIN_GR ? q.nb : -1;
    I.step = 0;
}

template <class T>
int ensure_dev(T *&p, size_t &cap, size_t count)
{
    if (count <= cap && p) return IMIN_OK;
    dfree(p);
    cap = 0;
    if (!ok(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)))) {
        (void)hipGetLastError();
        return IMIN_ENOMEM;
    }
    cap = count;
    return IMIN_OK;
}

void server_free(imin_server *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    multi_free(s->ms);
    dfree(s->d_table);
    dfree(s->d_stages);
    dfree(s->d_stage);
    dfree(s->d_rounds);
    dfree(s->d_out);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Admit queued queries, in arrival order, while their state fits: copy the graph's
// thresholds into each, then put seeds and bitmap in place and mask their in-edges.
int admit(imin_server *s)
{
    imin_graph *g = s->g;
    std::vector<Query> fresh;
    while (!s->queue.empty() &&
           (int32_t)(s->active.size() + fresh.size()) < s->cfg.max_active) {
        Query &q = s->queue.front();
        const size_t off = s->pool.alloc(q.bytes);
        if (off == SIZE_MAX) break;  // the head waits for memory; no overtaking
        q.off = off;
        carve(s, q);
        fresh.push_back(std::move(q));
        s->queue.pop_front();
    }
    if (fresh.empty()) return IMIN_OK;
    s->table.clear();
    s->stages.clear();
    s->stage.clear();
    const size_t quads = (size_t)std::max<int64_t>(((int64_t)g->m + 3) / 4, 1);
    for (Query &q : fresh) {
        if (!ok(hipMemcpyAsync(q.desc.thr4, g->d_thr_orig, quads * sizeof(uint4),
                               hipMemcpyDeviceToDevice, s->stream)))
            return IMIN_EDEVICE;
        imin::BatchStage st{};
        st.seeds = (int64_t)s->stage.size();
        s->stage.insert(s->stage.end(), q.seeds.begin(), q.seeds.end());
        st.bits = (int64_t)s->stage.size();
        st.words = (int32_t)q.inelig.size();
        for (uint32_t w : q.inelig) s->stage.push_back((int32_t)w);
        st.prev = (int64_t)s->stage.size();
        st.nprev = 0;
        st.now = (int64_t)s->stage.size();
        st.nnow = (int32_t)q.seeds.size();
        s->stage.insert(s->stage.end(), q.seeds.begin(), q.seeds.end());
        st.cand = -1;
        if (q.mode == IMIN_GR) {
            st.cand = (int64_t)s->stage.size();
            for (uint32_t w : q.cand) s->stage.push_back((int32_t)w);
        }
        s->stages.push_back(st);
        s->table.push_back(q.desc);
    }
    int rc = ensure_dev(s->d_stage, s->stage_cap, s->stage.size());
    if (rc) return rc;
    if (!ok(hipMemcpyAsync(s->d_table, s->table.data(), s->table.size() * sizeof(s->table[0]),
                           hipMemcpyHostToDevice, s->stream)) ||
        !ok(hipMemcpyAsync(s->d_stages, s->stages.data(),
                           s->stages.size() * sizeof(s->stages[0]), hipMemcpyHostToDevice,
                           s->stream)) ||
        !ok(hipMemcpyAsync(s->d_stage, s->stage.data(), s->stage.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s->stream)) ||
        !ok(imin::launch_batch_setup(s->d_table, s->d_stages, s->d_stage,
                                     (int32_t)fresh.size(), s->stream)) ||
        !ok(hipStreamSynchronize(s->stream)))
        return IMIN_EDEVICE;
    for (Query &q : fresh) s->active.push_back(std::move(q));
    return IMIN_OK;
}

// Retire the queries whose rounds are all done: gather their blockers and counters.
int retire(imin_server *s)
{
    std::vector<size_t> fin;
    for (size_t i = 0; i < s->active.size(); ++i)
        if (s->active[i].round >= s->active[i].rounds) fin.push_back(i);
    if (fin.empty()) return IMIN_OK;
    int32_t max_rounds = 1;
    s->table.clear();
    s->rounds.clear();
    for (size_t i : fin) {
        s->table.push_back(s->active[i].desc);
        s->rounds.push_back(s->active[i].nb);
        max_rounds = std::max(max_rounds, s->active[i].nb);
    }
    const int32_t stride = imin::kGatherB + max_rounds;
    const size_t k = fin.size();
    s->out.assign(k * (size_t)stride, 0);
    int rc = ensure_dev(s->d_out, s->out_cap, s->out.size());
    if (rc) return rc;
    if (!ok(hipMemcpyAsync(s->d_table, s->table.data(), k * sizeof(s->table[0]),
                           hipMemcpyHostToDevice, s->stream)) ||
        !ok(hipMemcpyAsync(s->d_rounds, s->rounds.data(), k * sizeof(int32_t),
                           hipMemcpyHostToDevice, s->stream)) ||
        !ok(imin::launch_batch_gather(s->d_table, s->d_rounds, s->d_out, stride, (int32_t)k,
                                      s->stream)) ||
        !ok(hipMemcpyAsync(s->out.data(), s->d_out, s->out.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s->stream)) ||
        !ok(hipStreamSynchronize(s->stream)))
        return IMIN_EDEVICE;
    for (size_t t = 0; t < k; ++t) {
        Query &q = s->active[fin[t]];
        const int32_t *o = s->out.data() + t * (size_t)stride;
        if (o[imin::kGatherErr] != 0) return IMIN_EDEVICE;
        Result r;
        r.B.assign(o + imin::kGatherB, o + imin::kGatherB + q.nb);
        for (int32_t v : r.B)
            if (v < 0) return IMIN_EDEVICE;
        unsigned long long st[kStats];
        for (int j = 0; j < kStats; ++j)
            st[j] = (unsigned long long)(uint32_t)o[2 * j] |
                    ((unsigned long long)(uint32_t)o[2 * j + 1] << 32);
        r.stats.samples = st[0];
        r.stats.reached = st[1];
        r.stats.edges_scanned = st[2];
        r.stats.live_edges = st[3];
        r.stats.spilled = st[4];
        r.stats.wave_samples = st[5];
        r.stats.pack_samples = st[6];
        s->done[q.ticket] = std::move(r);
        s->pending.erase(q.ticket);
        s->completed.push_back(q.ticket);
        s->pool.release(q.off, q.bytes);
    }
    std::vector<Query> keep;
    for (size_t i = 0; i < s->active.size(); ++i)
        if (s->active[i].round < s->active[i].rounds) keep.push_back(std::move(s->active[i]));
    s->active.swap(keep);
    return IMIN_OK;
}

}  // namespace

extern "C" {

int imin_server_create(imin_graph *g, const imin_server_config *cfg, imin_server **out)
{
    if (!g || !out) return IMIN_EINVAL;
    imin_server_config c{};
    if (cfg) c = *cfg;
    if (c.max_active < 0 || !launch_ok(&c.launch)) return IMIN_EINVAL;
    if (c.max_active == 0) c.max_active = kDefaultMaxActive;
    if (c.max_theta == 0) c.max_theta = kDefaultMaxTheta;
    if ((uint64_t)c.max_active * c.max_theta > kMaxTheta) return IMIN_ERANGE;
    if (!ok(hipSetDevice(g->device))) return IMIN_EDEVICE;
    if (c.hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (!ok(hipMemGetInfo(&free_b, &total_b))) return IMIN_EDEVICE;
        c.hbm_budget = free_b / 4;
    }
    imin_server *s = new (std::nothrow) imin_server();
    if (!s) return IMIN_ENOMEM;
    s->g = g;
    s->cfg = c;
    if (!ok(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking))) {
        server_free(s);
        return IMIN_EDEVICE;
    }
    if (!s->pool.init((size_t)c.hbm_budget)) {
        server_free(s);
        return IMIN_ENOMEM;
    }
    int rc = multi_alloc(s->ms, g->num_cus, g->n, g->m, (uint32_t)c.max_active * c.max_theta,
                         c.max_active, s->stream);
    size_t cap = 0;
    if (!rc) rc = ensure_dev(s->d_table, cap, (size_t)c.max_active);
    cap = 0;
    if (!rc) rc = ensure_dev(s->d_stages, cap, (size_t)c.max_active);
    cap = 0;
    if (!rc) rc = ensure_dev(s->d_rounds, cap, (size_t)c.max_active);
    if (!rc && !ok(hipStreamSynchronize(s->stream))) rc = IMIN_EDEVICE;
    if (rc) {
        server_free(s);
        return rc;
    }
    *out = s;
    return IMIN_OK;
}

void imin_server_destroy(imin_server *s) { server_free(s); }

int imin_server_query_bytes(const imin_server *s, int32_t nS, int32_t b, uint64_t *bytes)
{
    if (!s || !bytes || nS < 0 || b < 0) return IMIN_EINVAL;
    *bytes = footprint(s->g, nS, b);
    return IMIN_OK;
}

int imin_server_submit(imin_server *s, const int32_t *S, int32_t nS, int32_t b, uint32_t theta,
                       uint64_t seed, uint64_t *ticket)
{
    return imin_server_submit_mode(s, S, nS, b, theta, seed, IMIN_AG, ticket);
}

int imin_server_submit_mode(imin_server *s, const int32_t *S, int32_t nS, int32_t b,
                            uint32_t theta, uint64_t seed, int mode, uint64_t *ticket)
{
    if (!s || !ticket || theta == 0 || b < 0) return IMIN_EINVAL;
    if (mode != IMIN_AG && mode != IMIN_GR) return IMIN_EINVAL;
    if (theta > s->cfg.max_theta) return IMIN_ERANGE;
    Query q;
    int rc = seed_setup(s->g, S, nS, q.seeds, q.inelig);
    if (rc) return rc;
    q.b = b;
    q.mode = mode;
    if (mode == IMIN_GR) {
        q.nb = std::min(gr_candidates(s->g, q.seeds, q.inelig, q.cand), b);
        q.rounds = 2 * q.nb;
    } else {
        q.rounds = std::min<int32_t>(b, s->g->n - (int32_t)q.seeds.size());
        q.nb = q.rounds;
    }
    q.theta = theta;
    q.seed = seed;
    q.bytes = footprint(s->g, (int32_t)q.seeds.size(), b);
    if (align_up(q.bytes) > s->pool.size()) return IMIN_ERANGE;
    q.ticket = s->next_ticket++;
    *ticket = q.ticket;
    s->pending.insert(q.ticket);
    s->queue.push_back(std::move(q));
    return IMIN_OK;
}

int imin_server_step(imin_server *s, int32_t *n_active, int32_t *n_queued)
{
    if (!s) return IMIN_EINVAL;
    if (!ok(hipSetDevice(s->g->device))) return IMIN_EDEVICE;
    int rc = admit(s);
    if (rc) return rc;
    rc = retire(s);  // queries with no rounds at all
    if (rc) return rc;
    if (!s->active.empty()) {
        // one greedy round of every active query: key seed + round, its greedy round r
        s->table.clear();
        uint32_t total = 0;
        bool gr = false;
        for (Query &q : s->active) {
            imin::InstanceDesc I = q.desc;
            const uint64_t key = q.seed + (uint64_t)q.round;
            I.seed_lo = (uint32_t)key;
            I.seed_hi = (uint32_t)(key >> 32);
            I.step = q.round;
            I.sample_base = total;
            total += q.theta;
            s->table.push_back(I);
            gr = gr || q.mode == IMIN_GR;
        }
        if (!ok(hipMemcpyAsync(s->d_table, s->table.data(),
                               s->table.size() * sizeof(s->table[0]), hipMemcpyHostToDevice,
                               s->stream)))
            return IMIN_EDEVICE;
        rc = multi_round(s->ms, s->d_table, (int32_t)s->active.size(), total, 0u, s->cfg.launch,
                         s->g->num_cus, true, gr, s->g->model == IMIN_LT, s->stream);
        if (rc) return rc;
        // GreedyReplace queries whose replacement pass stopped this step end now
        const size_t na = s->active.size();
        if (gr) {
            rc = ensure_dev(s->d_out, s->out_cap, na);
            if (rc) return rc;
            s->out.assign(na, 0);
            if (!ok(imin::launch_batch_done(s->d_table, (int32_t)na,
                                            reinterpret_cast<uint32_t *>(s->d_out), s->stream)) ||
                !ok(hipMemcpyAsync(s->out.data(), s->d_out, na * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s->stream)))
                return IMIN_EDEVICE;
        }
        uint32_t wave_err = 0, wg_err = 0;
        rc = multi_errors(s->ms, &wave_err, &wg_err, s->stream);  // waits for the step
        if (rc) return rc;
        if (wave_err || wg_err) return IMIN_EDEVICE;
        for (size_t i = 0; i < na; ++i) {
            Query &q = s->active[i];
            ++q.round;
            if (gr && s->out[i] != 0) q.round = q.rounds;
        }
        rc = retire(s);
        if (rc) return rc;
    }
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return IMIN_OK;
}

int imin_server_completed(imin_server *s, uint64_t *tickets, int32_t cap, int32_t *count)
{
    if (!s || !count || cap < 0 || (cap > 0 && !tickets)) return IMIN_EINVAL;
    const int32_t k = std::min<int32_t>(cap, (int32_t)s->completed.size());
    std::copy(s->completed.begin(), s->completed.begin() + k, tickets);
    s->completed.erase(s->completed.begin(), s->completed.begin() + k);
    *count = k;
    return IMIN_OK;
}

int imin_server_result(imin_server *s, uint64_t ticket, int32_t *blockers, int32_t cap,
                       int32_t *n_blockers, imin_stats *stats)
{
    if (!s || !n_blockers || cap < 0 || (cap > 0 && !blockers)) return IMIN_EINVAL;
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return s->pending.count(ticket) ? 1 : IMIN_EINVAL;
    const Result &r = it->second;
    if ((int32_t)r.B.size() > cap) return IMIN_ERANGE;
    std::copy(r.B.begin(), r.B.end(), blockers);
    *n_blockers = (int32_t)r.B.size();
    if (stats) *stats = r.stats;
    s->done.erase(it);
    return IMIN_OK;
}

}  // extern "C"
