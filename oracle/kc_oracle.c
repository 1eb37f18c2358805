/*
 * kc_oracle.c -- CPU oracle for the 2-forest-sampling Kemeny-constant
 * estimator (Li, Liao, Li, Wang, "Scalable and Provable Kemeny Constant
 * Computation on Static and Dynamic Graphs: A 2-Forest Sampling Approach",
 * arXiv 2511.16356).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference the GPU library is checked against.  It shares no code, header,
 * table or helper with the GPU library; only tests, the package smoke check
 * and the benchmark's CPU-baseline leg may load it.
 *
 * What it computes, and where the paper defines it:
 *   - graph preparation: root = highest-degree vertex (section 5, Exp-III),
 *     BFS tree tau0 rooted there (Alg. 1, "Generate tau0 using BFS"), and
 *     tau0's depth-first numbering in/out (Alg. 1; section 3.2,
 *     "Depth-First Numbering");
 *   - Wilson's uniform-spanning-tree sampler (section 2.2 and Alg. 1), with
 *     each (sample, vertex, visit-count) drawing its neighbour from a
 *     Philox4x32-10 stream, so the sampled tree equals the cycle-popping
 *     result and does not depend on the walk order;
 *   - the per-tree value f(tau) of Theorem 3.3 in three independent forms:
 *       F1 naive       : the definition in Theorem 3.3 (compare each vertex's
 *                        tree path with its fixed tau0 path);
 *       F3 per edge    : the two sums of Theorem 3.4, each intersection
 *                        counted by brute force (the default form);
 *       F4 tau0 walk   : the O(n * depth) form mentioned in the proof of
 *                        Theorem 3.5 (walk each vertex's tau0 path and test
 *                        tree ancestry);
 *   - the estimator of Theorem 3.3, kappa = sum f / (2 m omega), returned to
 *     the caller as exact per-sample integers.
 *
 * Readings of the paper (where it is silent or misprinted):
 *   - Ties for the root go to the smallest vertex index; the BFS parent of v
 *     is its smallest-index neighbour one level closer to the root.
 *   - Algorithm 1 (a depth-first search over tau with a Fenwick tree over
 *     tau0's numbering) is not reproduced here: it is one way to evaluate
 *     the sums of Theorem 3.4, and the forms above evaluate the same sums
 *     directly from their definitions.
 *   - The random arrow: Philox4x32-10 (Salmon et al., SC'11) with counter
 *     (k, v, s_lo, s_hi) and key (seed_lo, seed_hi); outputs o0, o1 form
 *     x = o0 | o1 << 32, and the neighbour slot is floor(x * deg / 2^64).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ Philox4x32-10 */

#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

/* One Philox4x32 round: two 32x32->64 products, then the S-box style
 * permutation-and-xor with the round key. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)PH_M0 * c[0];
    uint64_t p1 = (uint64_t)PH_M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += PH_W0; k[1] += PH_W1; }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* The neighbour slot drawn by vertex v on its k-th visit in sample s. */
uint32_t orc_arrow(uint64_t seed, uint64_t s, uint32_t v, uint32_t k, uint32_t deg) {
    uint32_t ctr[4] = {k, v, (uint32_t)s, (uint32_t)(s >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox(ctr, key, o);
    uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    unsigned __int128 prod = (unsigned __int128)x * deg;
    return (uint32_t)(prod >> 64);
}

/* ------------------------------------------------------- graph preparation */

enum { ORC_OK = 0, ORC_INVALID = 1, ORC_DISCONNECTED = 2, ORC_NOMEM = 3, ORC_LIMIT = 6 };

/*
 * Root, BFS tree tau0 and its numbering.
 *   root   : given (>= 0) or highest degree, smallest index on ties;
 *   dist   : BFS distance from root;
 *   p0     : smallest-index neighbour u with dist(u) = dist(v) - 1 (-1 at root);
 *   in0    : preorder position in a DFS of tau0 visiting children in ascending
 *            index order; out0 = largest preorder position in v's subtree.
 */
int orc_prepare(int64_t n, const int64_t *off, const int32_t *adj, int32_t root_in,
                int32_t *root_out, int32_t *p0, int32_t *dist, int32_t *in0,
                int32_t *out0, int32_t *depth_out) {
    if (n < 2) return ORC_INVALID;
    int32_t root = root_in;
    if (root < 0) {
        int64_t best = -1;
        for (int64_t v = 0; v < n; ++v) {
            int64_t d = off[v + 1] - off[v];
            if (d > best) { best = d; root = (int32_t)v; }
        }
    }
    if (root < 0 || root >= n) return ORC_INVALID;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return ORC_NOMEM;
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    int64_t qh = 0, qt = 0;
    dist[root] = 0;
    queue[qt++] = root;
    while (qh < qt) {
        int32_t x = queue[qh++];
        for (int64_t e = off[x]; e < off[x + 1]; ++e) {
            int32_t y = adj[e];
            if (dist[y] < 0) { dist[y] = dist[x] + 1; queue[qt++] = y; }
        }
    }
    if (qt != n) { free(queue); return ORC_DISCONNECTED; }
    int32_t depth = 0;
    for (int64_t v = 0; v < n; ++v) {
        p0[v] = -1;
        if (dist[v] > depth) depth = dist[v];
        if (v == root) continue;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = adj[e];
            if (dist[u] == dist[v] - 1 && (p0[v] < 0 || u < p0[v])) p0[v] = u;
        }
    }
    /* children of tau0 in ascending order: counting sort by parent, then by
     * scanning v ascending the children lists are ascending automatically. */
    int64_t *cstart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *clist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *cfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *spos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!cstart || !clist || !cfill || !spos) { free(queue); free(cstart); free(clist); free(cfill); free(spos); return ORC_NOMEM; }
    for (int64_t v = 0; v < n; ++v) if (p0[v] >= 0) cstart[p0[v] + 1]++;
    for (int64_t v = 0; v < n; ++v) cstart[v + 1] += cstart[v];
    for (int64_t v = 0; v < n; ++v) cfill[v] = cstart[v];
    for (int64_t v = 0; v < n; ++v) if (p0[v] >= 0) clist[cfill[p0[v]]++] = (int32_t)v;
    /* iterative DFS: queue[] reused as the stack, spos = next child index */
    int64_t sp = 0, t = 0;
    queue[sp++] = root;
    in0[root] = (int32_t)t++;
    spos[root] = cstart[root];
    while (sp > 0) {
        int32_t x = queue[sp - 1];
        if (spos[x] < cstart[x + 1]) {
            int32_t c = clist[spos[x]++];
            in0[c] = (int32_t)t++;
            spos[c] = cstart[c];
            queue[sp++] = c;
        } else {
            out0[x] = (int32_t)(t - 1);
            sp--;
        }
    }
    free(queue); free(cstart); free(clist); free(cfill); free(spos);
    *root_out = root;
    *depth_out = depth;
    return ORC_OK;
}

/* ------------------------------------------------------------ Wilson's UST */

/*
 * Wilson's algorithm: from each vertex not yet in the tree, run a random walk
 * until it meets the tree, then add the loop-erased path.  The walk at x on
 * its cnt[x]-th draw goes to adj[off[x] + arrow(seed, s, x, cnt[x])].  The
 * last draw at each vertex is its tree parent, so parent[] and cnt[] are
 * exactly the cycle-popping outcome of those arrow stacks.
 *
 * order: start vertices (NULL = ascending).  Returns total draws, or -1 when
 * max_steps (> 0) is exceeded.
 */
int64_t orc_wilson(int64_t n, const int64_t *off, const int32_t *adj, int32_t root,
                   uint64_t seed, uint64_t s, const int32_t *order, int64_t max_steps,
                   int32_t *parent, uint32_t *cnt, uint8_t *intree) {
    for (int64_t v = 0; v < n; ++v) { cnt[v] = 0; intree[v] = 0; parent[v] = -1; }
    intree[root] = 1;
    int64_t steps = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t u = order ? order[i] : (int32_t)i;
        int32_t x = u;
        while (!intree[x]) {
            uint32_t deg = (uint32_t)(off[x + 1] - off[x]);
            uint32_t j = orc_arrow(seed, s, (uint32_t)x, cnt[x], deg);
            cnt[x]++;
            parent[x] = adj[off[x] + j];
            x = parent[x];
            if (max_steps > 0 && ++steps > max_steps) return -1;
            if (max_steps <= 0) ++steps;
        }
        x = u;
        while (!intree[x]) { intree[x] = 1; x = parent[x]; }
    }
    parent[root] = -1;
    return steps;
}

/* ------------------------------------------------- per-tree helper arrays */

typedef struct {
    int64_t n, two_m;
    const int64_t *off;
    int32_t root;
    const int32_t *p0, *in0, *out0, *parent;
    /* derived from parent: */
    int64_t *vol;     /* vol(Sub(tau, v)) */
    int32_t *tin, *tout; /* tau preorder interval */
    int64_t *cstart;  /* tau children lists */
    int32_t *clist;
    int32_t *stack;
    int64_t *spos;
} tree_ctx;

static int64_t deg_of(const tree_ctx *t, int64_t v) { return t->off[v + 1] - t->off[v]; }

/* children lists of tau, a preorder numbering, and subtree volumes (summed in
 * reverse preorder, so every child is finished before its parent). */
static int tree_build(tree_ctx *t) {
    int64_t n = t->n;
    t->vol = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t->tin = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    t->tout = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    t->cstart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    t->clist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    t->stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    t->spos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!t->vol || !t->tin || !t->tout || !t->cstart || !t->clist || !t->stack || !t->spos || !order) {
        free(order);
        return ORC_NOMEM;
    }
    for (int64_t v = 0; v < n; ++v) if (v != t->root) t->cstart[t->parent[v] + 1]++;
    for (int64_t v = 0; v < n; ++v) t->cstart[v + 1] += t->cstart[v];
    for (int64_t v = 0; v < n; ++v) t->spos[v] = t->cstart[v];
    for (int64_t v = 0; v < n; ++v) if (v != t->root) t->clist[t->spos[t->parent[v]]++] = (int32_t)v;
    int64_t sp = 0, k = 0;
    t->stack[sp++] = t->root;
    t->spos[t->root] = t->cstart[t->root];
    order[k] = t->root;
    t->tin[t->root] = (int32_t)k++;
    while (sp > 0) {
        int32_t x = t->stack[sp - 1];
        if (t->spos[x] < t->cstart[x + 1]) {
            int32_t c = t->clist[t->spos[x]++];
            t->spos[c] = t->cstart[c];
            order[k] = c;
            t->tin[c] = (int32_t)k++;
            t->stack[sp++] = c;
        } else {
            t->tout[x] = (int32_t)(k - 1);
            sp--;
        }
    }
    if (k != n) { free(order); return ORC_INVALID; } /* parent[] is not a tree */
    for (int64_t v = 0; v < n; ++v) t->vol[v] = deg_of(t, v);
    for (int64_t i = n - 1; i > 0; --i) {
        int32_t v = order[i];
        t->vol[t->parent[v]] += t->vol[v];
    }
    free(order);
    return ORC_OK;
}

static void tree_free(tree_ctx *t) {
    free(t->vol); free(t->tin); free(t->tout); free(t->cstart); free(t->clist);
    free(t->stack); free(t->spos);
}

static int is_tau_anc(const tree_ctx *t, int32_t a, int32_t v) {
    return t->tin[a] <= t->tin[v] && t->tin[v] <= t->tout[a];
}

static int is_tau0_anc(const tree_ctx *t, int32_t a, int32_t v) {
    return t->in0[a] <= t->in0[v] && t->in0[v] <= t->out0[a];
}

/* ---------------------------------------------------- f(tau): four forms */

/*
 * F1 -- Theorem 3.3 as stated.  For each u != r: mark the directed edges of
 * the fixed path P_u (u's path to r in tau0), then walk u's path to r in tau.
 * An edge (w -> parent(w)) of the tree path that is also an edge of P_u in
 * the same direction yields the 2-forest tau \ (w, parent(w)) in the forward
 * set; in the opposite direction, in the reverse set.  Its r-side tree is
 * V \ Sub(tau, w), of volume 2m - vol(Sub(tau, w)).
 */
static int64_t f_naive(tree_ctx *t) {
    int64_t n = t->n;
    /* mark[x] = u  <=>  x lies on P_u (so the directed edge x -> p0(x) is in P_u) */
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) mark[v] = -1;
    int64_t f = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (u == t->root) continue;
        for (int32_t x = (int32_t)u; x != t->root; x = t->p0[x]) mark[x] = (int32_t)u;
        int64_t acc = 0;
        for (int32_t w = (int32_t)u; w != t->root; w = t->parent[w]) {
            int32_t pw = t->parent[w];
            int64_t volT1 = t->two_m - t->vol[w];
            if (mark[w] == u && t->p0[w] == pw) acc += volT1;          /* same direction */
            else if (mark[pw] == u && t->p0[pw] == w) acc -= volT1;    /* opposite direction */
        }
        f += deg_of(t, u) * acc;
    }
    free(mark);
    return f;
}

/*
 * F3 -- Theorem 3.4: f = sum over tree edges (v, p(v)) oriented like tau0 of
 * (2m - vol(Sub(tau,v))) * vol(Sub(tau,v) & Sub(tau0,v)), minus the sum over
 * tree edges oriented against tau0 of (2m - vol(Sub(tau,v))) *
 * vol(Sub(tau,v) & Sub(tau0,p(v))).  Intersections are counted by brute force
 * over the tau0 subtree's preorder range.
 */
static int64_t f_peredge(tree_ctx *t) {
    int64_t n = t->n;
    int32_t *at0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n); /* vertex at tau0 preorder i */
    for (int64_t v = 0; v < n; ++v) at0[t->in0[v]] = (int32_t)v;
    int64_t f = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (v == t->root) continue;
        int32_t pv = t->parent[v];
        int32_t top;
        int64_t sign;
        if (t->p0[v] == pv) { top = (int32_t)v; sign = 1; }
        else if (t->p0[pv] == v) { top = pv; sign = -1; }
        else continue;
        int64_t inter = 0;
        for (int32_t i = t->in0[top]; i <= t->out0[top]; ++i) {
            int32_t u = at0[i];
            if (is_tau_anc(t, (int32_t)v, u)) inter += deg_of(t, u);
        }
        f += sign * (t->two_m - t->vol[v]) * inter;
    }
    free(at0);
    return f;
}

/*
 * F4 -- walk each y's tau0 path: at the tau0 edge (x -> p0(x)) add
 * +(2m - vol(x)) if parent(x) = p0(x) and x is a tau-ancestor of y; add
 * -(2m - vol(p0(x))) if p0(x) != r, parent(p0(x)) = x and p0(x) is a
 * tau-ancestor of y.  f = sum_y d(y) * q(y).
 */
static int64_t f_walk(tree_ctx *t) {
    int64_t f = 0;
    for (int64_t y = 0; y < t->n; ++y) {
        int64_t q = 0;
        for (int32_t x = (int32_t)y; x != t->root; x = t->p0[x]) {
            int32_t z = t->p0[x];
            if (t->parent[x] == z && is_tau_anc(t, x, (int32_t)y)) q += t->two_m - t->vol[x];
            if (z != t->root && t->parent[z] == x && is_tau_anc(t, z, (int32_t)y)) q -= t->two_m - t->vol[z];
        }
        f += deg_of(t, y) * q;
    }
    return f;
}

enum { F_NAIVE = 1, F_PEREDGE = 3, F_WALK = 4 };

/*
 * f(tau) for a given rooted spanning tree.  p0/in0/out0 describe the fixed
 * tree tau0 (any spanning tree rooted at `root`, not only the BFS one).
 * Returns ORC_OK and writes *f_out, or an error code when parent[] is not a
 * spanning tree rooted at root.
 */
int orc_f(int64_t n, const int64_t *off, int32_t root, const int32_t *p0, const int32_t *in0,
          const int32_t *out0, const int32_t *parent, int form, int64_t *f_out) {
    tree_ctx t;
    memset(&t, 0, sizeof(t));
    t.n = n; t.off = off; t.two_m = off[n]; t.root = root;
    t.p0 = p0; t.in0 = in0; t.out0 = out0; t.parent = parent;
    if (parent[root] != -1) return ORC_INVALID;
    for (int64_t v = 0; v < n; ++v)
        if (v != root && (parent[v] < 0 || parent[v] >= n)) return ORC_INVALID;
    int st = tree_build(&t);
    if (st != ORC_OK) { tree_free(&t); return st; }
    int64_t f = 0;
    switch (form) {
        case F_NAIVE: f = f_naive(&t); break;
        case F_PEREDGE: f = f_peredge(&t); break;
        case F_WALK: f = f_walk(&t); break;
        default: tree_free(&t); return ORC_INVALID;
    }
    tree_free(&t);
    *f_out = f;
    return ORC_OK;
}

/* ---------------------------------------------------------- batch drivers */

typedef struct {
    int64_t n; const int64_t *off; const int32_t *adj; int32_t root;
    const int32_t *p0, *in0, *out0;
    uint64_t seed; int64_t s_begin, s_end, s0; int form; int64_t max_steps;
    int64_t *f_out; int64_t *steps_out;
    int32_t *parents_out; uint32_t *cnt_out; /* sample mode */
    const int64_t *ids;                       /* optional list of sample ids */
    int status;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    int64_t n = j->n;
    /* sample ids: s_begin..s_end-1, or ids[s_begin..s_end-1] when a list is given */
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *cnt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint8_t *intree = (uint8_t *)malloc((size_t)n);
    j->status = ORC_OK;
    for (int64_t t = j->s_begin; t < j->s_end && j->status == ORC_OK; ++t) {
        int64_t s = j->ids ? j->ids[t - j->s0] : t;
        int64_t steps = orc_wilson(n, j->off, j->adj, j->root, j->seed, (uint64_t)s, NULL,
                                   j->max_steps, parent, cnt, intree);
        int64_t i = t - j->s0;
        if (steps < 0) { j->status = ORC_LIMIT; break; }
        if (j->steps_out) j->steps_out[i] = steps;
        if (j->parents_out) {
            memcpy(j->parents_out + i * n, parent, sizeof(int32_t) * (size_t)n);
            if (j->cnt_out) memcpy(j->cnt_out + i * n, cnt, sizeof(uint32_t) * (size_t)n);
        }
        if (j->f_out) {
            int64_t f;
            int st = orc_f(n, j->off, j->root, j->p0, j->in0, j->out0, parent, j->form, &f);
            if (st != ORC_OK) { j->status = st; break; }
            j->f_out[i] = f;
        }
    }
    free(parent); free(cnt); free(intree);
    return NULL;
}

static int run_batch(job_t *proto, int64_t s0, int64_t count, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > count) nthreads = (int)(count > 0 ? count : 1);
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int i = 0; i < nthreads; ++i) {
        jobs[i] = *proto;
        jobs[i].s0 = s0;
        jobs[i].s_begin = s0 + count * i / nthreads;
        jobs[i].s_end = s0 + count * (i + 1) / nthreads;
        pthread_create(&th[i], NULL, run_job, &jobs[i]);
    }
    int status = ORC_OK;
    for (int i = 0; i < nthreads; ++i) {
        pthread_join(th[i], NULL);
        if (jobs[i].status != ORC_OK) status = jobs[i].status;
    }
    free(jobs); free(th);
    return status;
}

/* Samples s0 .. s0+count-1: parents [count*n] (root -> -1) and draw counts. */
int orc_sample(int64_t n, const int64_t *off, const int32_t *adj, int32_t root, uint64_t seed,
               int64_t s0, int64_t count, int nthreads, int64_t max_steps,
               int32_t *parents_out, uint32_t *cnt_out, int64_t *steps_out) {
    job_t j;
    memset(&j, 0, sizeof(j));
    j.n = n; j.off = off; j.adj = adj; j.root = root; j.seed = seed; j.max_steps = max_steps;
    j.parents_out = parents_out; j.cnt_out = cnt_out; j.steps_out = steps_out;
    return run_batch(&j, s0, count, nthreads);
}

/* Samples s0 .. s0+count-1: per-sample f (form F1..F4) and draw totals. */
int orc_estimate(int64_t n, const int64_t *off, const int32_t *adj, int32_t root,
                 const int32_t *p0, const int32_t *in0, const int32_t *out0, uint64_t seed,
                 int64_t s0, int64_t count, int nthreads, int form, int64_t max_steps,
                 int64_t *f_out, int64_t *steps_out) {
    job_t j;
    memset(&j, 0, sizeof(j));
    j.n = n; j.off = off; j.adj = adj; j.root = root; j.p0 = p0; j.in0 = in0; j.out0 = out0;
    j.seed = seed; j.form = form; j.max_steps = max_steps; j.f_out = f_out; j.steps_out = steps_out;
    return run_batch(&j, s0, count, nthreads);
}

/* Per-sample f (form F1, F3 or F4) and draw totals for the sample ids ids[0..count-1]. */
int orc_estimate_ids(int64_t n, const int64_t *off, const int32_t *adj, int32_t root,
                     const int32_t *p0, const int32_t *in0, const int32_t *out0, uint64_t seed,
                     const int64_t *ids, int64_t count, int nthreads, int form, int64_t max_steps,
                     int64_t *f_out, int64_t *steps_out) {
    job_t j;
    memset(&j, 0, sizeof(j));
    j.n = n; j.off = off; j.adj = adj; j.root = root; j.p0 = p0; j.in0 = in0; j.out0 = out0;
    j.seed = seed; j.form = form; j.max_steps = max_steps; j.f_out = f_out; j.steps_out = steps_out;
    j.ids = ids;
    return run_batch(&j, 0, count, nthreads);
}

/* Wilson with an explicit start order (for the order-independence pin). */
/*
 * Wilson's algorithm with the two vertices u and v both in the tree from the
 * start (section 4.1: a uniform spanning tree that contains the new edge
 * (u, v) is the edge plus a uniform spanning forest of two trees rooted at
 * u and v).  Same arrows as orc_wilson; walks start in ascending order.
 * parent[u] = parent[v] = -1 on return.  Returns total draws.
 */
int orc_wilson_two_roots(int64_t n, const int64_t *off, const int32_t *adj, int32_t u, int32_t v,
                         uint64_t seed, uint64_t s, int32_t *parent, uint32_t *cnt, int64_t *steps_out) {
    uint8_t *intree = (uint8_t *)malloc((size_t)n);
    if (!intree) return ORC_NOMEM;
    for (int64_t x = 0; x < n; ++x) { cnt[x] = 0; intree[x] = 0; parent[x] = -1; }
    intree[u] = 1;
    intree[v] = 1;
    int64_t steps = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t x = (int32_t)i;
        while (!intree[x]) {
            uint32_t deg = (uint32_t)(off[x + 1] - off[x]);
            uint32_t j = orc_arrow(seed, s, (uint32_t)x, cnt[x], deg);
            cnt[x]++;
            parent[x] = adj[off[x] + j];
            x = parent[x];
            ++steps;
        }
        x = (int32_t)i;
        while (!intree[x]) { intree[x] = 1; x = parent[x]; }
    }
    parent[u] = -1;
    parent[v] = -1;
    free(intree);
    *steps_out = steps;
    return ORC_OK;
}

int orc_wilson_order(int64_t n, const int64_t *off, const int32_t *adj, int32_t root,
                     uint64_t seed, uint64_t s, const int32_t *order,
                     int32_t *parent, uint32_t *cnt, int64_t *steps_out) {
    uint8_t *intree = (uint8_t *)malloc((size_t)n);
    int64_t st = orc_wilson(n, off, adj, root, seed, s, order, 0, parent, cnt, intree);
    free(intree);
    *steps_out = st;
    return ORC_OK;
}
