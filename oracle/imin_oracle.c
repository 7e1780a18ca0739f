/*
 * imin_oracle.c -- plain CPU oracle for the live-edge spread-decrease estimate and the two
 * greedy drivers built on it. Each sample is computed by one thread; the _mt entry points
 * only split a call's independent samples over host threads and add their integer sums.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library path may link, load or call this
 * file; it exists so tests, the smoke check and the benchmark's CPU-baseline leg can
 * compare the GPU results against an implementation that is slow but easy to audit.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * What it computes (citations are to arXiv 2302.13529):
 *   - IC model and blockers: Section III-A, Definition 2 (a blocked vertex never activates).
 *   - Multiple seeds are merged into one source (Section V, "From Multiple Seeds to One
 *     Seed"). Here the merged source is a virtual root r whose edge to v is live iff at
 *     least one seed->v edge is live; this has the same law as the paper's 1-prod(1-p_i)
 *     edge and needs no floating-point product.
 *   - A random sampled graph keeps each edge e=(u,v) independently with probability p
 *     (Definition 4). Its coin is a Philox4x32-10 word (Salmon et al., SC'11):
 *        w = Philox4x32_10(counter=(e>>2, j, 0, 0), key=(lo32(k), hi32(k)))[e & 3]
 *        live(j, e)  <=>  (w >> 8) < ceil(p * 2^24)       (p >= 1 -> always live)
 *     where j is the sample index and k = seed + call index of the greedy driver.
 *     Only edges leaving vertices reachable from r are ever decided: the dominator tree
 *     of a sampled graph depends only on its part reachable from r.
 *   - Per sample: dominator tree by Lengauer-Tarjan over a DFS numbering from the source
 *     (Section V-B3, Lemma 3), subtree sizes c[u] by a DFS of that tree, and
 *     Delta[u] += c[u] (Algorithm 2). Delta is kept as the exact integer sum
 *     D[u] = sum_j c_j[u]; Delta = D / theta is never formed, so the argmax of the
 *     greedy drivers never depends on summation order.
 *   - AdvancedGreedy (Algorithm 3) and GreedyReplace (Algorithm 4); ties in the argmax go
 *     to the smallest vertex id, seeds are never candidates.
 *   - Triggering model (Section V-E), as the linear-threshold instance: the weight w(v,u) of
 *     each in-edge of u (sum over u's in-edges <= 1) is the probability that v alone forms
 *     u's triggering set; with the remaining probability the set is empty. A sampled graph
 *     keeps exactly the in-edge of u named by u's triggering set. u's choice in sample j:
 *        R = Philox4x32_10(counter=(u>>2, j, 1, 0), key)[u & 3] >> 8
 *        bound_k = min(2^24, ceil(2^24 * (w_1 + ... + w_k)))   (fp64 running sums over u's
 *                  in-edges taken in ascending edge id; bound_0 = 0)
 *        the in-edge e_k with bound_{k-1} <= R < bound_k, or none when R >= bound_last.
 *     Everything downstream (dominators, counts, greedy) is unchanged.
 *
 * Parity pins live in tests/: Philox against torch's header-only engine, the coin rule
 * against the float test over all 2^24 values, dominators against networkx and against
 * vertex-deletion brute force (Theorem 6), the estimator against exact enumeration of all
 * live-edge worlds (Lemma 1, Theorem 4) and the paper's toy-graph numbers (Examples 1-4,
 * Table III), the greedy drivers against brute-force greedy on deterministic graphs.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_IC 0
#define ORC_LT 1

/* ---------------------------------------------------------------- Philox4x32-10 */

static uint32_t mul_hi32(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

/* One Philox4x32 round followed by nothing else; the key schedule is applied by the caller. */
static void philox_round(uint32_t x[4], uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint32_t hi0 = mul_hi32(M0, x[0]), lo0 = M0 * x[0];
    uint32_t hi1 = mul_hi32(M1, x[2]), lo1 = M1 * x[2];
    uint32_t y0 = hi1 ^ x[1] ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k1;
    uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        philox_round(x, k0, k1);
        k0 += W0;
        k1 += W1;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* ---------------------------------------------------------------- coin rule */

/* ceil(p * 2^24) for p in [0, 1]; p * 2^24 is exact in fp32 (a power-of-two scale). */
uint32_t orc_threshold(float p)
{
    if (!(p > 0.0f)) return 0u;
    if (p >= 1.0f) return 1u << 24;
    return (uint32_t)ceilf(p * 16777216.0f);
}

static int edge_live(uint64_t key, uint32_t j, int64_t e, uint32_t thr)
{
    uint32_t ctr[4] = {(uint32_t)(e >> 2), j, 0u, 0u};
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, k, w);
    return (w[e & 3] >> 8) < thr;
}

int orc_edge_live(uint64_t key, uint32_t j, int64_t e, float p)
{
    return edge_live(key, j, e, orc_threshold(p));
}

/* Upper end of an in-edge's 24-bit interval from the fp64 running sum of the weights up to
 * and including that edge: min(2^24, ceil(2^24 * sum)). */
static double lt_bound(double sum)
{
    double bound = ceil(sum * 16777216.0);
    return bound > 16777216.0 ? 16777216.0 : bound;
}

/* LT: the in-edge of u chosen in sample j (its triggering set), or -1 for none. */
static int64_t lt_trigger(const int32_t *in_ptr, const int32_t *in_edge, const float *w,
                          uint64_t key, uint32_t j, int32_t u)
{
    uint32_t ctr[4] = {(uint32_t)u >> 2, j, 1u, 0u};
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, k, out);
    const double R = (double)(out[u & 3] >> 8);
    double sum = 0.0;
    for (int32_t i = in_ptr[u]; i < in_ptr[u + 1]; ++i) {
        sum += (double)w[in_edge[i]];
        if (R < lt_bound(sum)) return in_edge[i];
    }
    return -1;
}

/* ---------------------------------------------------------------- problem state */

typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    int model;             /* ORC_IC or ORC_LT */
    const float *w;        /* LT: edge weights */
    int32_t *in_ptr, *in_edge; /* LT: in-edges of each vertex, ascending edge id */
    int64_t *trig;         /* LT: the choice of each vertex in the current sample ... */
    uint64_t *trig_tag;    /* ... valid when its tag equals the sample's tag */
    uint64_t tag;
    uint32_t *thr;         /* per edge */
    uint8_t *is_seed;      /* per vertex */
    const uint8_t *blocked;/* per vertex, may be NULL */
    int32_t *seeds;        /* distinct seeds, ascending */
    int32_t nseeds;

    /* per-sample scratch, sized to n+1 vertices / the edges actually met */
    int32_t *loc;          /* global id -> local id, -1 when unreached (reset after use) */
    int32_t *glob;         /* local id -> global id; local 0 is the virtual root */
    int32_t nloc;
    int32_t *esrc, *edst;  /* live edges of the reached part, local ids */
    int64_t nedge, cap_edge;
    /* CSR of successors / predecessors over local ids */
    int32_t *succ_ptr, *succ, *pred_ptr, *pred;
    /* Lengauer-Tarjan arrays over DFS numbers */
    int32_t *num, *vert, *parent, *semi, *idom, *ancestor, *label, *stack, *bucket_head, *bucket_next;
    int32_t *size, *child_ptr, *child, *fill;
    uint64_t edges_scanned, live_edges;
} orc_state;

static int live_in_sample(orc_state *st, uint64_t key, uint32_t j, int64_t e)
{
    if (st->model == ORC_LT) {
        /* each vertex's choice is drawn once per sample and remembered for the sample */
        int32_t u = st->col[e];
        if (st->trig_tag[u] != st->tag) {
            st->trig[u] = lt_trigger(st->in_ptr, st->in_edge, st->w, key, j, u);
            st->trig_tag[u] = st->tag;
        }
        return st->trig[u] == e;
    }
    return edge_live(key, j, e, st->thr[e]);
}

static int blocked_at(const orc_state *st, int32_t v)
{
    return st->blocked ? st->blocked[v] != 0 : 0;
}

static int eligible(const orc_state *st, int32_t v)
{
    return !st->is_seed[v] && !blocked_at(st, v);
}

static int push_edge(orc_state *st, int32_t a, int32_t b)
{
    if (st->nedge == st->cap_edge) {
        int64_t cap = st->cap_edge ? 2 * st->cap_edge : 1024;
        int32_t *s2 = (int32_t *)realloc(st->esrc, (size_t)cap * sizeof(int32_t));
        if (!s2) return ORC_ENOMEM;
        st->esrc = s2;
        int32_t *d2 = (int32_t *)realloc(st->edst, (size_t)cap * sizeof(int32_t));
        if (!d2) return ORC_ENOMEM;
        st->edst = d2;
        st->cap_edge = cap;
    }
    st->esrc[st->nedge] = a;
    st->edst[st->nedge] = b;
    st->nedge++;
    return ORC_OK;
}

static int32_t visit(orc_state *st, int32_t v)
{
    if (st->loc[v] < 0) {
        st->loc[v] = st->nloc;
        st->glob[st->nloc] = v;
        st->nloc++;
    }
    return st->loc[v];
}

/*
 * Reached part of sampled graph j: the virtual root (local 0), every vertex reachable
 * from it over live edges whose target is neither a seed nor blocked, and every live
 * edge among them. Edges into seeds are dropped: the merged source has no incoming
 * edges that matter (Section V, multiple seeds to one seed).
 */
static int build_sample(orc_state *st, uint64_t key, uint32_t j)
{
    st->tag++;  /* a new sample: forget the remembered choices */
    st->nloc = 0;
    st->nedge = 0;
    st->glob[0] = -1;
    st->nloc = 1;
    for (int32_t i = 0; i < st->nseeds; ++i) {
        int32_t s = st->seeds[i];
        for (int64_t e = st->row_ptr[s]; e < st->row_ptr[s + 1]; ++e) {
            int32_t v = st->col[e];
            st->edges_scanned++;
            if (!live_in_sample(st, key, j, e)) continue;
            if (!eligible(st, v)) continue;
            st->live_edges++;
            int32_t lv = visit(st, v);
            if (push_edge(st, 0, lv)) return ORC_ENOMEM;
        }
    }
    for (int32_t q = 1; q < st->nloc; ++q) {   /* nloc grows while we scan: BFS queue */
        int32_t u = st->glob[q];
        for (int64_t e = st->row_ptr[u]; e < st->row_ptr[u + 1]; ++e) {
            int32_t v = st->col[e];
            st->edges_scanned++;
            if (!live_in_sample(st, key, j, e)) continue;
            if (!eligible(st, v)) continue;
            st->live_edges++;
            int32_t lv = visit(st, v);
            if (push_edge(st, q, lv)) return ORC_ENOMEM;
        }
    }
    return ORC_OK;
}

static void build_adjacency(orc_state *st)
{
    int32_t N = st->nloc;
    memset(st->succ_ptr, 0, (size_t)(N + 1) * sizeof(int32_t));
    memset(st->pred_ptr, 0, (size_t)(N + 1) * sizeof(int32_t));
    for (int64_t i = 0; i < st->nedge; ++i) {
        st->succ_ptr[st->esrc[i] + 1]++;
        st->pred_ptr[st->edst[i] + 1]++;
    }
    for (int32_t v = 0; v < N; ++v) {
        st->succ_ptr[v + 1] += st->succ_ptr[v];
        st->pred_ptr[v + 1] += st->pred_ptr[v];
    }
    for (int32_t v = 0; v < N; ++v) st->fill[v] = st->succ_ptr[v];
    for (int64_t i = 0; i < st->nedge; ++i) st->succ[st->fill[st->esrc[i]]++] = st->edst[i];
    for (int32_t v = 0; v < N; ++v) st->fill[v] = st->pred_ptr[v];
    for (int64_t i = 0; i < st->nedge; ++i) st->pred[st->fill[st->edst[i]]++] = st->esrc[i];
}

/* Iterative depth-first search from local 0: DFS numbers, vertex of each number, parent. */
static void dfs_number(orc_state *st)
{
    int32_t N = st->nloc;
    for (int32_t v = 0; v < N; ++v) st->num[v] = -1;
    int32_t count = 0, top = 0;
    /* stack holds vertices; fill[v] is the next successor index of v still to try */
    st->num[0] = count;
    st->vert[count] = 0;
    st->parent[count] = -1;
    count++;
    st->fill[0] = st->succ_ptr[0];
    st->stack[top++] = 0;
    while (top > 0) {
        int32_t v = st->stack[top - 1];
        if (st->fill[v] == st->succ_ptr[v + 1]) { top--; continue; }
        int32_t w = st->succ[st->fill[v]++];
        if (st->num[w] >= 0) continue;
        st->num[w] = count;
        st->vert[count] = w;
        st->parent[count] = st->num[v];
        count++;
        st->fill[w] = st->succ_ptr[w];
        st->stack[top++] = w;
    }
}

/* Path compression of the Lengauer-Tarjan forest, written without recursion. */
static void lt_compress(orc_state *st, int32_t v)
{
    int32_t top = 0;
    int32_t x = v;
    while (st->ancestor[st->ancestor[x]] >= 0) {
        st->stack[top++] = x;
        x = st->ancestor[x];
    }
    while (top > 0) {
        int32_t y = st->stack[--top];
        int32_t a = st->ancestor[y];
        if (st->semi[st->label[a]] < st->semi[st->label[y]]) st->label[y] = st->label[a];
        st->ancestor[y] = st->ancestor[a];
    }
}

static int32_t lt_eval(orc_state *st, int32_t v)
{
    if (st->ancestor[v] < 0) return v;
    lt_compress(st, v);
    return st->label[v];
}

/*
 * Lengauer-Tarjan over DFS numbers 0..N-1 (0 = source). On return idom[w] holds the DFS
 * number of the immediate dominator of DFS number w (idom[0] = -1).
 * Semidominators are minima over DFS paths; idom follows from Lemma 3, with the
 * "otherwise" case resolved in a final pass in increasing DFS order.
 */
static void lengauer_tarjan(orc_state *st)
{
    int32_t N = st->nloc;
    for (int32_t w = 0; w < N; ++w) {
        st->semi[w] = w;
        st->ancestor[w] = -1;
        st->label[w] = w;
        st->bucket_head[w] = -1;
        st->idom[w] = -1;
    }
    for (int32_t w = N - 1; w >= 1; --w) {
        int32_t lw = st->vert[w];
        for (int32_t k = st->pred_ptr[lw]; k < st->pred_ptr[lw + 1]; ++k) {
            int32_t v = st->num[st->pred[k]];
            int32_t u = lt_eval(st, v);
            if (st->semi[u] < st->semi[w]) st->semi[w] = st->semi[u];
        }
        /* bucket[semi[w]] += w */
        st->bucket_next[w] = st->bucket_head[st->semi[w]];
        st->bucket_head[st->semi[w]] = w;
        int32_t p = st->parent[w];
        st->ancestor[w] = p;                       /* link(parent[w], w) */
        for (int32_t v = st->bucket_head[p]; v >= 0; v = st->bucket_next[v]) {
            int32_t u = lt_eval(st, v);
            st->idom[v] = (st->semi[u] < st->semi[v]) ? u : p;
        }
        st->bucket_head[p] = -1;
    }
    for (int32_t w = 1; w < N; ++w)
        if (st->idom[w] != st->semi[w]) st->idom[w] = st->idom[st->idom[w]];
    st->idom[0] = -1;
}

/* Subtree sizes of the dominator tree by an iterative post-order DFS from the source. */
static void subtree_sizes(orc_state *st)
{
    int32_t N = st->nloc;
    memset(st->child_ptr, 0, (size_t)(N + 1) * sizeof(int32_t));
    for (int32_t w = 1; w < N; ++w) st->child_ptr[st->idom[w] + 1]++;
    for (int32_t w = 0; w < N; ++w) st->child_ptr[w + 1] += st->child_ptr[w];
    for (int32_t w = 0; w < N; ++w) st->fill[w] = st->child_ptr[w];
    for (int32_t w = 1; w < N; ++w) st->child[st->fill[st->idom[w]]++] = w;
    for (int32_t w = 0; w < N; ++w) { st->size[w] = 1; st->fill[w] = st->child_ptr[w]; }
    int32_t top = 0;
    st->stack[top++] = 0;
    while (top > 0) {
        int32_t v = st->stack[top - 1];
        if (st->fill[v] < st->child_ptr[v + 1]) {
            st->stack[top++] = st->child[st->fill[v]++];
        } else {
            top--;
            if (top > 0) st->size[st->stack[top - 1]] += st->size[v];
        }
    }
}

static void state_free(orc_state *st)
{
    free(st->thr); free(st->is_seed); free(st->seeds); free(st->in_ptr); free(st->in_edge);
    free(st->trig); free(st->trig_tag);
    free(st->loc); free(st->glob); free(st->esrc); free(st->edst);
    free(st->succ_ptr); free(st->succ); free(st->pred_ptr); free(st->pred);
    free(st->num); free(st->vert); free(st->parent); free(st->semi); free(st->idom);
    free(st->ancestor); free(st->label); free(st->stack); free(st->bucket_head);
    free(st->bucket_next); free(st->size); free(st->child_ptr); free(st->child); free(st->fill);
    memset(st, 0, sizeof(*st));
}

static int check_graph(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob)
{
    if (n <= 0 || !row_ptr) return ORC_EINVAL;
    if (row_ptr[0] != 0) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_EINVAL;
    int64_t m = row_ptr[n];
    if (m > 0 && (!col || !prob)) return ORC_EINVAL;
    for (int64_t e = 0; e < m; ++e) {
        if (col[e] < 0 || col[e] >= n) return ORC_EINVAL;
        if (!(prob[e] >= 0.0f && prob[e] <= 1.0f)) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* In-edges of every vertex in ascending edge id (a counting sort by target). */
static int build_in_edges(orc_state *st, int64_t m)
{
    int32_t n = st->n;
    st->in_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    st->in_edge = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!st->in_ptr || !st->in_edge || !fill) { free(fill); return ORC_ENOMEM; }
    for (int64_t e = 0; e < m; ++e) st->in_ptr[st->col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) st->in_ptr[v + 1] += st->in_ptr[v];
    for (int32_t v = 0; v < n; ++v) fill[v] = st->in_ptr[v];
    for (int64_t e = 0; e < m; ++e) st->in_edge[fill[st->col[e]]++] = (int32_t)e;
    free(fill);
    return ORC_OK;
}

/* LT weights: the in-edge weights of every vertex sum to at most 1 (up to fp32 rounding). */
static int check_lt_weights(const orc_state *st)
{
    for (int32_t v = 0; v < st->n; ++v) {
        double sum = 0.0;
        for (int32_t i = st->in_ptr[v]; i < st->in_ptr[v + 1]; ++i) sum += st->w[st->in_edge[i]];
        if (sum > 1.0 + 1e-5) return ORC_EINVAL;
    }
    return ORC_OK;
}

static int state_init(orc_state *st, int32_t n, const int32_t *row_ptr, const int32_t *col,
                      const float *prob, const int32_t *S, int32_t nS, int model)
{
    memset(st, 0, sizeof(*st));
    if (model != ORC_IC && model != ORC_LT) return ORC_EINVAL;
    int rc = check_graph(n, row_ptr, col, prob);
    if (rc) return rc;
    if (nS <= 0 || !S) return ORC_EINVAL;
    for (int32_t i = 0; i < nS; ++i)
        if (S[i] < 0 || S[i] >= n) return ORC_EINVAL;
    int64_t m = row_ptr[n];
    st->n = n;
    st->row_ptr = row_ptr;
    st->col = col;
    size_t N1 = (size_t)n + 2;
    st->thr = (uint32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint32_t));
    st->is_seed = (uint8_t *)calloc((size_t)n, 1);
    st->seeds = (int32_t *)malloc((size_t)nS * sizeof(int32_t));
#define ALLOC_I32(f) st->f = (int32_t *)malloc(N1 * sizeof(int32_t))
    ALLOC_I32(loc); ALLOC_I32(glob); ALLOC_I32(succ_ptr); ALLOC_I32(pred_ptr);
    ALLOC_I32(num); ALLOC_I32(vert); ALLOC_I32(parent); ALLOC_I32(semi); ALLOC_I32(idom);
    ALLOC_I32(ancestor); ALLOC_I32(label); ALLOC_I32(stack); ALLOC_I32(bucket_head);
    ALLOC_I32(bucket_next); ALLOC_I32(size); ALLOC_I32(child_ptr); ALLOC_I32(child); ALLOC_I32(fill);
#undef ALLOC_I32
    if (!st->thr || !st->is_seed || !st->seeds || !st->loc || !st->glob || !st->succ_ptr ||
        !st->pred_ptr || !st->num || !st->vert || !st->parent || !st->semi || !st->idom ||
        !st->ancestor || !st->label || !st->stack || !st->bucket_head || !st->bucket_next ||
        !st->size || !st->child_ptr || !st->child || !st->fill) {
        state_free(st);
        return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < m; ++e) st->thr[e] = orc_threshold(prob[e]);
    st->model = model;
    st->w = prob;
    if (model == ORC_LT) {
        rc = build_in_edges(st, m);
        if (!rc) rc = check_lt_weights(st);
        if (!rc) {
            st->trig = (int64_t *)malloc((size_t)n * sizeof(int64_t));
            st->trig_tag = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
            if (!st->trig || !st->trig_tag) rc = ORC_ENOMEM;
        }
        if (rc) { state_free(st); return rc; }
    }
    for (int32_t i = 0; i < nS; ++i) st->is_seed[S[i]] = 1;
    st->nseeds = 0;
    for (int32_t v = 0; v < n; ++v)
        if (st->is_seed[v]) st->seeds[st->nseeds++] = v;
    for (int32_t v = 0; v < n; ++v) st->loc[v] = -1;
    return ORC_OK;
}

static int ensure_edge_arrays(orc_state *st)
{
    /* succ / pred must hold nedge entries */
    size_t need = (size_t)(st->nedge > 0 ? st->nedge : 1);
    int32_t *a = (int32_t *)realloc(st->succ, need * sizeof(int32_t));
    if (!a) return ORC_ENOMEM;
    st->succ = a;
    int32_t *b = (int32_t *)realloc(st->pred, need * sizeof(int32_t));
    if (!b) return ORC_ENOMEM;
    st->pred = b;
    return ORC_OK;
}

/*
 * One sampled graph: fills c_local (size per local id via st->size, indexed by DFS number)
 * and returns through the state. After the call st->vert / st->size / st->glob describe it.
 */
static int one_sample(orc_state *st, uint64_t key, uint32_t j)
{
    int rc = build_sample(st, key, j);
    if (rc) return rc;
    rc = ensure_edge_arrays(st);
    if (rc) return rc;
    build_adjacency(st);
    dfs_number(st);
    lengauer_tarjan(st);
    subtree_sizes(st);
    return ORC_OK;
}

static void reset_loc(orc_state *st)
{
    for (int32_t q = 1; q < st->nloc; ++q) st->loc[st->glob[q]] = -1;
}

static int check_blocked(const orc_state *st)
{
    if (!st->blocked) return ORC_OK;
    for (int32_t v = 0; v < st->n; ++v)
        if (st->blocked[v] && st->is_seed[v]) return ORC_EINVAL;  /* B is a subset of V \ S */
    return ORC_OK;
}

/*
 * Sample j alone: c_out[v] = size of v's dominator subtree (0 if v is unreached),
 * idom_out[v] = global id of idom(v) (-1 for children of the merged source, -2 if v is
 * unreached or a seed). Returns |R_j| (reached non-seed vertices) or a negative error.
 */
int64_t orc_sample_m(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                     const int32_t *S, int32_t nS, const uint8_t *blocked, uint64_t key,
                     uint32_t j, int32_t *c_out, int32_t *idom_out, int model)
{
    orc_state st;
    int rc = state_init(&st, n, row_ptr, col, prob, S, nS, model);
    if (rc) return rc;
    st.blocked = blocked;
    rc = check_blocked(&st);
    if (rc) { state_free(&st); return rc; }
    rc = one_sample(&st, key, j);
    if (rc) { state_free(&st); return rc; }
    for (int32_t v = 0; v < n; ++v) {
        if (c_out) c_out[v] = 0;
        if (idom_out) idom_out[v] = -2;
    }
    for (int32_t w = 1; w < st.nloc; ++w) {
        int32_t g = st.glob[st.vert[w]];
        if (c_out) c_out[g] = st.size[w];
        if (idom_out) idom_out[g] = st.glob[st.vert[st.idom[w]]];
    }
    int64_t r = st.nloc - 1;
    reset_loc(&st);
    state_free(&st);
    return r;
}

/* stats[0] samples, [1] reached (sum of |R_j|), [2] edges scanned, [3] live edges taken */
static int decrease_into(orc_state *st, uint32_t theta, uint64_t key, uint64_t *counts,
                         uint64_t *stats)
{
    for (int32_t v = 0; v < st->n; ++v) counts[v] = 0;
    uint64_t reached = 0;
    st->edges_scanned = 0;
    st->live_edges = 0;
    for (uint32_t j = 0; j < theta; ++j) {
        int rc = one_sample(st, key, j);
        if (rc) return rc;
        for (int32_t w = 1; w < st->nloc; ++w)
            counts[st->glob[st->vert[w]]] += (uint64_t)st->size[w];
        reached += (uint64_t)(st->nloc - 1);
        reset_loc(st);
    }
    if (stats) {
        stats[0] = theta;
        stats[1] = reached;
        stats[2] = st->edges_scanned;
        stats[3] = st->live_edges;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- threaded variant */

/*
 * Algorithm 2 draws its sampled graphs independently of one another and only adds integers
 * into the counts, so the samples may run on several host threads, in any order, with the
 * same result. Thread t of T takes the samples j = t, t + T, t + 2T, ... with a scratch
 * state and uint64 counts of its own; counts and work counters are summed once every thread
 * is done. A pool of one thread is decrease_into itself. This variant exists to check large
 * configurations in reasonable time; tests pin it equal to the single-threaded function.
 */
#define ORC_MAX_THREADS 256

typedef struct {
    orc_state *st;
    uint32_t theta, t, T;
    uint64_t key;
    uint64_t *counts;   /* n entries, this thread's own */
    uint64_t stats[4];
    int rc;
} mt_part;

static void *mt_part_run(void *arg)
{
    mt_part *p = (mt_part *)arg;
    orc_state *st = p->st;
    for (int32_t v = 0; v < st->n; ++v) p->counts[v] = 0;
    uint64_t reached = 0, samples = 0;
    st->edges_scanned = 0;
    st->live_edges = 0;
    p->rc = ORC_OK;
    for (uint64_t j = p->t; j < p->theta; j += p->T) {
        int rc = one_sample(st, p->key, (uint32_t)j);
        if (rc) { p->rc = rc; return NULL; }
        for (int32_t w = 1; w < st->nloc; ++w)
            p->counts[st->glob[st->vert[w]]] += (uint64_t)st->size[w];
        reached += (uint64_t)(st->nloc - 1);
        samples++;
        reset_loc(st);
    }
    p->stats[0] = samples;
    p->stats[1] = reached;
    p->stats[2] = st->edges_scanned;
    p->stats[3] = st->live_edges;
    return NULL;
}

typedef struct {
    int T;
    orc_state *st;    /* T states over the same problem */
    uint64_t *part;   /* (T - 1) * n counts of threads 1 .. T-1 */
} orc_pool;

static void pool_free(orc_pool *pl)
{
    if (pl->st)
        for (int t = 0; t < pl->T; ++t) state_free(&pl->st[t]);
    free(pl->st);
    free(pl->part);
    memset(pl, 0, sizeof(*pl));
}

static int pool_init(orc_pool *pl, int T, int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const float *prob, const int32_t *S, int32_t nS, int model)
{
    memset(pl, 0, sizeof(*pl));
    if (T < 1 || T > ORC_MAX_THREADS) return ORC_EINVAL;
    pl->st = (orc_state *)calloc((size_t)T, sizeof(orc_state));
    if (!pl->st) return ORC_ENOMEM;
    for (int t = 0; t < T; ++t) {
        int rc = state_init(&pl->st[t], n, row_ptr, col, prob, S, nS, model);
        if (rc) { pl->T = t; pool_free(pl); return rc; }
        pl->T = t + 1;
    }
    if (T > 1) {
        pl->part = (uint64_t *)malloc((size_t)(T - 1) * (size_t)n * sizeof(uint64_t));
        if (!pl->part) { pool_free(pl); return ORC_ENOMEM; }
    }
    return ORC_OK;
}

static void pool_set_blocked(orc_pool *pl, const uint8_t *blocked)
{
    for (int t = 0; t < pl->T; ++t) pl->st[t].blocked = blocked;
}

/* Algorithm 2 on the pool's threads: the same counts and stats as decrease_into. */
static int pool_decrease(orc_pool *pl, uint32_t theta, uint64_t key, uint64_t *counts,
                         uint64_t *stats)
{
    uint32_t T = (uint32_t)pl->T < theta ? (uint32_t)pl->T : theta;
    if (T <= 1) return decrease_into(&pl->st[0], theta, key, counts, stats);
    const int32_t n = pl->st[0].n;
    mt_part parts[ORC_MAX_THREADS];
    pthread_t th[ORC_MAX_THREADS];
    int started[ORC_MAX_THREADS];
    for (uint32_t t = 0; t < T; ++t) {
        memset(&parts[t], 0, sizeof(parts[t]));
        parts[t].st = &pl->st[t];
        parts[t].theta = theta;
        parts[t].t = t;
        parts[t].T = T;
        parts[t].key = key;
        parts[t].counts = t == 0 ? counts : pl->part + (size_t)(t - 1) * (size_t)n;
        started[t] = 0;
    }
    int rc = ORC_OK;
    for (uint32_t t = 1; t < T; ++t) {
        if (pthread_create(&th[t], NULL, mt_part_run, &parts[t]) != 0) { rc = ORC_ENOMEM; break; }
        started[t] = 1;
    }
    if (!rc) mt_part_run(&parts[0]);
    for (uint32_t t = 1; t < T; ++t)
        if (started[t]) pthread_join(th[t], NULL);
    if (rc) return rc;
    uint64_t tot[4] = {0, 0, 0, 0};
    for (uint32_t t = 0; t < T; ++t) {
        if (parts[t].rc) return parts[t].rc;
        for (int k = 0; k < 4; ++k) tot[k] += parts[t].stats[k];
    }
    for (uint32_t t = 1; t < T; ++t) {
        const uint64_t *c = parts[t].counts;
        for (int32_t v = 0; v < n; ++v) counts[v] += c[v];
    }
    if (stats)
        for (int k = 0; k < 4; ++k) stats[k] = tot[k];
    return ORC_OK;
}

/* Algorithm 2 as orc_decrease_m, its samples spread over nthreads host threads. */
int orc_decrease_mt(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                    const int32_t *S, int32_t nS, const uint8_t *blocked, uint32_t theta,
                    uint64_t key, uint64_t *counts, uint64_t *stats, int model, int nthreads)
{
    if (theta == 0 || !counts) return ORC_EINVAL;
    orc_pool pl;
    int rc = pool_init(&pl, nthreads, n, row_ptr, col, prob, S, nS, model);
    if (rc) return rc;
    pool_set_blocked(&pl, blocked);
    rc = check_blocked(&pl.st[0]);
    if (!rc) rc = pool_decrease(&pl, theta, key, counts, stats);
    pool_free(&pl);
    return rc;
}

int64_t orc_sample(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                   const int32_t *S, int32_t nS, const uint8_t *blocked, uint64_t key,
                   uint32_t j, int32_t *c_out, int32_t *idom_out)
{
    return orc_sample_m(n, row_ptr, col, prob, S, nS, blocked, key, j, c_out, idom_out, ORC_IC);
}

/* Algorithm 2 with integer accumulation: counts[u] = sum over theta samples of c_j[u]. */
int orc_decrease_m(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                   const int32_t *S, int32_t nS, const uint8_t *blocked, uint32_t theta,
                   uint64_t key, uint64_t *counts, uint64_t *stats, int model)
{
    if (theta == 0 || !counts) return ORC_EINVAL;
    orc_state st;
    int rc = state_init(&st, n, row_ptr, col, prob, S, nS, model);
    if (rc) return rc;
    st.blocked = blocked;
    rc = check_blocked(&st);
    if (!rc) rc = decrease_into(&st, theta, key, counts, stats);
    state_free(&st);
    return rc;
}

int orc_decrease(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                 const int32_t *S, int32_t nS, const uint8_t *blocked, uint32_t theta,
                 uint64_t key, uint64_t *counts, uint64_t *stats)
{
    return orc_decrease_m(n, row_ptr, col, prob, S, nS, blocked, theta, key, counts, stats,
                          ORC_IC);
}

/* LT: the in-edge chosen by u in sample j under key (its triggering set), or -1. */
int64_t orc_lt_trigger(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *w,
                       uint64_t key, uint32_t j, int32_t u)
{
    if (u < 0 || u >= n) return ORC_EINVAL;
    orc_state st;
    memset(&st, 0, sizeof(st));
    if (check_graph(n, row_ptr, col, w)) return ORC_EINVAL;
    st.n = n;
    st.row_ptr = row_ptr;
    st.col = col;
    st.w = w;
    if (build_in_edges(&st, row_ptr[n])) { state_free(&st); return ORC_ENOMEM; }
    int64_t e = lt_trigger(st.in_ptr, st.in_edge, w, key, j, u);
    state_free(&st);
    return e;
}

/* LT: the interval upper ends bound_1, bound_2, ... of u's in-edges in ascending edge id
 * (the values lt_trigger compares against), written to bounds[]; returns their count. */
int64_t orc_lt_bounds(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *w,
                      int32_t u, uint32_t *bounds)
{
    if (u < 0 || u >= n || !bounds) return ORC_EINVAL;
    orc_state st;
    memset(&st, 0, sizeof(st));
    if (check_graph(n, row_ptr, col, w)) return ORC_EINVAL;
    st.n = n;
    st.row_ptr = row_ptr;
    st.col = col;
    if (build_in_edges(&st, row_ptr[n])) { state_free(&st); return ORC_ENOMEM; }
    double sum = 0.0;
    int64_t k = 0;
    for (int32_t i = st.in_ptr[u]; i < st.in_ptr[u + 1]; ++i) {
        sum += (double)w[st.in_edge[i]];
        bounds[k++] = (uint32_t)lt_bound(sum);
    }
    state_free(&st);
    return k;
}

#define ORC_AG 0
#define ORC_GR 1

/*
 * Greedy drivers. Call r (0, 1, 2, ...) of Algorithm 2 uses Philox key seed + r.
 *   AG (Algorithm 3): b rounds of argmax over V \ (S u B).
 *   GR (Algorithm 4): greedy over the out-neighbours of the merged seed, then a pass over
 *     a snapshot of the chosen blockers in reverse insertion order: unblock u, re-estimate,
 *     take the argmax x over V \ (S u B), put x in u's slot, stop when x == u.
 * blockers[] receives the slots in order; *n_blockers their count; calls_out the number
 * of calls of Algorithm 2 made; stats accumulate over all calls.
 */
int orc_greedy_mt(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                  const int32_t *S, int32_t nS, int32_t b, uint32_t theta, uint64_t seed,
                  int32_t mode, int32_t *blockers, int32_t *n_blockers, int32_t *calls_out,
                  uint64_t *stats, int model, int nthreads);

static int greedy_core(orc_pool *pl, const int32_t *row_ptr, const int32_t *col, int32_t b,
                       uint32_t theta, uint64_t seed, int32_t mode, int32_t *blockers,
                       int32_t *n_blockers, int32_t *calls_out, uint64_t *stats)
{
    orc_state *st = &pl->st[0];
    const int32_t n = st->n;
    uint64_t tot[4] = {0, 0, 0, 0}, one[4];
    uint64_t call = 0;
    int32_t nb = 0;
    int rc = ORC_OK;
    uint8_t *blk = (uint8_t *)calloc((size_t)n, 1);
    uint64_t *D = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint8_t *cand = (uint8_t *)calloc((size_t)n, 1);
    int32_t *B = (int32_t *)malloc((size_t)(b > 0 ? b : 1) * sizeof(int32_t));
    int32_t *snap = (int32_t *)malloc((size_t)(b > 0 ? b : 1) * sizeof(int32_t));
    if (!blk || !D || !cand || !B || !snap) { rc = ORC_ENOMEM; goto done; }
    pool_set_blocked(pl, blk);
    if (mode == ORC_AG) {
        int32_t nonseed = n - st->nseeds;
        int32_t rounds = b < nonseed ? b : nonseed;
        for (int32_t r = 0; r < rounds; ++r) {
            rc = pool_decrease(pl, theta, seed + call, D, one);
            if (rc) goto done;
            call++;
            for (int k = 0; k < 4; ++k) tot[k] += one[k];
            int32_t x = -1;
            for (int32_t u = 0; u < n; ++u) {
                if (st->is_seed[u] || blk[u]) continue;
                if (x == -1 || D[u] > D[x]) x = u;
            }
            blk[x] = 1;
            B[nb++] = x;
        }
    } else {
        /* CB = out-neighbours of the merged seed, seeds excluded */
        int32_t ncb = 0;
        for (int32_t i = 0; i < st->nseeds; ++i) {
            int32_t s = st->seeds[i];
            for (int64_t e = row_ptr[s]; e < row_ptr[s + 1]; ++e) {
                int32_t v = col[e];
                if (!st->is_seed[v] && !cand[v]) { cand[v] = 1; ncb++; }
            }
        }
        int32_t k = ncb < b ? ncb : b;
        for (int32_t r = 0; r < k; ++r) {
            rc = pool_decrease(pl, theta, seed + call, D, one);
            if (rc) goto done;
            call++;
            for (int q = 0; q < 4; ++q) tot[q] += one[q];
            int32_t x = -1;
            for (int32_t u = 0; u < n; ++u) {
                if (!cand[u]) continue;
                if (x == -1 || D[u] > D[x]) x = u;
            }
            cand[x] = 0;
            blk[x] = 1;
            B[nb++] = x;
        }
        memcpy(snap, B, (size_t)nb * sizeof(int32_t));
        for (int32_t i = nb - 1; i >= 0; --i) {
            int32_t u = snap[i];
            int32_t slot = -1;
            for (int32_t q = 0; q < nb; ++q)
                if (B[q] == u) slot = q;
            blk[u] = 0;
            rc = pool_decrease(pl, theta, seed + call, D, one);
            if (rc) goto done;
            call++;
            for (int q = 0; q < 4; ++q) tot[q] += one[q];
            int32_t x = -1;
            for (int32_t v = 0; v < n; ++v) {
                if (st->is_seed[v] || blk[v]) continue;
                if (x == -1 || D[v] > D[x]) x = v;
            }
            B[slot] = x;
            blk[x] = 1;
            if (x == u) break;
        }
    }
    memcpy(blockers, B, (size_t)nb * sizeof(int32_t));
    *n_blockers = nb;
    if (calls_out) *calls_out = (int32_t)call;
    if (stats) for (int q = 0; q < 4; ++q) stats[q] = tot[q];
    rc = ORC_OK;
done:
    pool_set_blocked(pl, NULL);
    free(blk); free(D); free(cand); free(B); free(snap);
    return rc;
}

int orc_greedy_m(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                 const int32_t *S, int32_t nS, int32_t b, uint32_t theta, uint64_t seed,
                 int32_t mode, int32_t *blockers, int32_t *n_blockers, int32_t *calls_out,
                 uint64_t *stats, int model)
{
    return orc_greedy_mt(n, row_ptr, col, prob, S, nS, b, theta, seed, mode, blockers,
                         n_blockers, calls_out, stats, model, 1);
}

/* The greedy drivers with every Algorithm 2 call spread over nthreads host threads. */
int orc_greedy_mt(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
                  const int32_t *S, int32_t nS, int32_t b, uint32_t theta, uint64_t seed,
                  int32_t mode, int32_t *blockers, int32_t *n_blockers, int32_t *calls_out,
                  uint64_t *stats, int model, int nthreads)
{
    if (theta == 0 || b < 0 || !blockers || !n_blockers) return ORC_EINVAL;
    if (mode != ORC_AG && mode != ORC_GR) return ORC_EINVAL;
    orc_pool pl;
    int rc = pool_init(&pl, nthreads, n, row_ptr, col, prob, S, nS, model);
    if (rc) return rc;
    rc = greedy_core(&pl, row_ptr, col, b, theta, seed, mode, blockers, n_blockers, calls_out,
                     stats);
    pool_free(&pl);
    return rc;
}

int orc_greedy(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *prob,
               const int32_t *S, int32_t nS, int32_t b, uint32_t theta, uint64_t seed,
               int32_t mode, int32_t *blockers, int32_t *n_blockers, int32_t *calls_out,
               uint64_t *stats)
{
    return orc_greedy_m(n, row_ptr, col, prob, S, nS, b, theta, seed, mode, blockers,
                        n_blockers, calls_out, stats, ORC_IC);
}
