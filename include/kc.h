/*
 * kc.h -- C ABI of the MI355X (gfx950) Kemeny-constant library.
 *
 * The library evaluates the 2-forest-sampling estimator of Li, Liao, Li and
 * Wang, "Scalable and Provable Kemeny Constant Computation on Static and
 * Dynamic Graphs: A 2-Forest Sampling Approach" (arXiv 2511.16356):
 *
 *     kappa(G) ~= (1 / (2 m omega)) * sum_{i=1..omega} f(tau_i)     (Theorem 3.3)
 *
 * where tau_i are uniform spanning trees drawn with Wilson's algorithm
 * (section 2.2; Algorithm 1) and f(tau) is the path-mapping value of
 * Theorem 3.3, evaluated per tree with the per-edge identity of Theorem 3.4
 * (subtree volumes over a fixed BFS tree tau0).  Every step after graph
 * preparation runs in HIP kernels on the GPU.
 *
 * Conventions shared by all calls
 *   - Every call returns a kc_status; nothing throws across the ABI.
 *     kc_last_error() gives a human-readable detail for the calling thread.
 *   - A graph is a simple, connected, undirected graph (section 2.1) given
 *     as CSR: row v lists the neighbours of v in strictly ascending order,
 *     each undirected edge appears in both rows, no self-loops.
 *   - "device pointer" means memory on the current HIP device (for example a
 *     torch CUDA tensor's data_ptr); "host pointer" means ordinary memory.
 *     The caller owns every array it passes; the library owns kc_graph.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue their kernels on it and return after the stream has
 *     finished the call's work, so outputs are ready on return.
 *   - Calls on one kc_graph must not overlap; different graphs are
 *     independent.
 *   - A sample is identified by its global index s (not its batch
 *     position): the tree of sample s is a pure function of (graph, root,
 *     seed, s), identical alone or in any batch, for any launch shape.
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KC_OK = 0,
    KC_ERR_INVALID = 1,      /* malformed CSR, bad argument, bad root, self-loop, duplicate */
    KC_ERR_DISCONNECTED = 2, /* the graph is not connected (section 2.1 requires it) */
    KC_ERR_NOMEM = 3,        /* device or host allocation failed */
    KC_ERR_DEVICE = 4,       /* a HIP runtime call failed */
    KC_ERR_OVERFLOW = 5,     /* 4 m^2 depth(tau0) >= 2^63, or 2m >= 2^31 (32-bit volumes) */
    KC_ERR_LIMIT = 6,        /* a sample exceeded the step limit; its results are discarded */
    KC_ERR_UNSUPPORTED = 7   /* a size outside what the kernels are built for */
} kc_status;

typedef struct kc_graph kc_graph;

/* Read-only facts about a prepared graph. */
typedef struct {
    int64_t n;          /* vertices */
    int64_t two_m;      /* sum of degrees = 2 |E| */
    int32_t root;       /* r: highest degree, smallest index on ties, unless given */
    int32_t depth0;     /* depth of tau0 (for the BFS rule: the eccentricity of r) */
    int32_t max_degree;
    int32_t traversal;  /* KC_TRAV_WALK or KC_TRAV_SWEEP, as chosen for this graph */
    int64_t device_bytes; /* graph arrays resident on the device */
    int32_t tau0;       /* KC_TAU0_* rule tau0 is built with */
    int64_t sample_bytes; /* device workspace one sample in flight needs in kc_estimate under the
                             current traversal (sampler state, tree numbering, sweep Fenwick tree) */
    int32_t chains;     /* walks one sample may hold open at once (KC_OPT_CHAINS) */
} kc_graph_info;

/* How tau0, the fixed spanning tree whose root paths define the path mapping,
 * is chosen (Theorem 3.4 holds for any spanning tree; section 5, Exp-II
 * compares breadth-first, depth-first and random trees). */
enum {
    KC_TAU0_BFS = 0,   /* breadth-first from r, parent = smallest-index neighbour one level up
                          (Algorithm 1; the default) */
    KC_TAU0_DFS = 1,   /* depth-first from r, rows scanned in ascending order, parent = the
                          vertex a vertex is discovered from */
    KC_TAU0_GIVEN = 2  /* a spanning tree the caller supplies (kc_set_tau0) */
};

/* Traversal variants for f(tau) (Theorem 3.4); results are identical. */
enum {
    KC_TRAV_AUTO = 0,
    KC_TRAV_WALK = 1,  /* per vertex, walk its tau0 ancestors: O(n depth0) per tree */
    KC_TRAV_SWEEP = 2  /* tau0-preorder sweep with a Fenwick tree over tau's volume-weighted
                          numbering: O(n log m) per tree (the paper's O(n log n) form) */
};

/* Options for kc_set_option. */
enum {
    KC_OPT_WALKERS = 1,    /* cooperating walkers per sample, 1..64 (default 64) */
    KC_OPT_SLOTS = 2,      /* samples in flight per launch (0 = sized from free HBM) */
    KC_OPT_TRAVERSAL = 3,  /* KC_TRAV_* */
    KC_OPT_STEP_LIMIT = 4, /* per-sample cap on sampler rounds (0 = default 1024 n + 2^22) */
    KC_OPT_MEM_BUDGET = 5, /* bytes of device workspace the library may allocate (0 = 80% of free) */
    KC_OPT_START_ORDER = 6, /* order in which walks are started (results do not depend on it):
                              0 = BFS order from the root, 1 = reverse BFS order,
                              2 = a fixed pseudo-random permutation (default) */
    KC_OPT_CHAINS = 7,     /* walks one sample may hold open at once: 1024 or 2048 (default:
                              2048 for graphs of at least 100,000 vertices and mean degree
                              below 4, else 1024).  More finish one sample in fewer rounds;
                              fewer let more samples run at once.  Results do not depend on it. */
    KC_OPT_MAINTENANCE = 8, /* KC_MAINT_*: how kc_apply_updates maintains the resident set;
                              may change while the set's weights are all equal (always under
                              basic maintenance), else KC_ERR_INVALID */
    KC_OPT_LEAN_LOOKS = 9  /* a walk's look at its next vertex is the claim alone, and a vertex
                              it claims has its arrow word and graph record read in the next
                              round (fewer lines where most looks meet the tree, one more
                              round per claim): 0 = when the mean degree is at least 8
                              (default), 1 = off, 2 = on.  Results do not depend on it. */
};

/* Sample maintenance of a resident set (section 4). */
enum {
    KC_MAINT_BASIC = 0,    /* Algorithm 2: replace trees by fresh uniform samples (default) */
    KC_MAINT_IMPROVED = 1  /* Algorithm 3: link-cut / cut-link the affected trees and weight them */
};

/*
 * Prepare a graph (Algorithm 1, "Generate tau0 using BFS" and the DFN of
 * tau0; root choice of section 5).  Validates the CSR, checks connectivity,
 * picks r, builds tau0 (BFS parent = smallest-index neighbour one level
 * closer to r) and tau0's preorder numbering, and copies everything the
 * kernels need to the device.
 *   n        : vertex count, >= 2
 *   offsets  : HOST pointer, n+1 entries, int64 if offsets_are_i64 else int32
 *   indices  : HOST pointer, offsets[n] int32 entries
 *   root     : -1 to choose automatically, else the root vertex
 *   out      : receives the handle (NULL on failure)
 * Errors: KC_ERR_INVALID, KC_ERR_DISCONNECTED, KC_ERR_OVERFLOW, KC_ERR_NOMEM,
 * KC_ERR_DEVICE, KC_ERR_UNSUPPORTED (max degree >= 2^20, or n > 2^31 - 1024).
 */
kc_status kc_graph_create(int64_t n, const void *offsets, int offsets_are_i64,
                          const int32_t *indices, int32_t root, void *hip_stream,
                          kc_graph **out);

/* Free the graph and its device workspace.  NULL is accepted. */
kc_status kc_graph_destroy(kc_graph *g);

/* Copy the graph's facts into *info (host pointer). */
kc_status kc_graph_get_info(const kc_graph *g, kc_graph_info *info);

/* Set a KC_OPT_* option.  KC_ERR_INVALID for an unknown option or value. */
kc_status kc_set_option(kc_graph *g, int option, int64_t value);

/*
 * Choose tau0 (KC_TAU0_*).  f(tau) changes with tau0 tree by tree, its mean
 * over uniform trees does not (Theorem 3.4); a tau0 with shorter root paths
 * gives a smaller variance (section 5, Exp-II).  Trees already drawn keep
 * their parent arrays; the resident set's f values are recomputed on the new
 * tau0.  Updates (kc_apply_updates) rebuild tau0 with the same rule on the new
 * graph; a given tree is kept while all its edges remain and gives way to
 * KC_TAU0_BFS when one of them is deleted.
 *   kind   : KC_TAU0_BFS, KC_TAU0_DFS or KC_TAU0_GIVEN
 *   parent : HOST pointer, n int32, read for KC_TAU0_GIVEN only (copied):
 *            parent[r] = -1 and, for every other v, (v, parent[v]) an edge of
 *            the graph, with every vertex reaching r
 * Errors: KC_ERR_INVALID (unknown kind; a given array that is not a spanning
 * tree of the graph rooted at r), KC_ERR_OVERFLOW (4 m^2 depth(tau0) >= 2^63),
 * KC_ERR_NOMEM, KC_ERR_DEVICE.  On an error nothing changes.
 */
kc_status kc_set_tau0(kc_graph *g, int kind, const int32_t *parent, void *hip_stream);

/*
 * Allocate, ahead of time, the device workspace that kc_estimate needs for
 * batches of up to `count` samples (per-sample sampler and traversal state
 * for the samples in flight, and the per-sample result buffers), so that a
 * later call allocates nothing.  Calls also allocate on first use when this
 * is skipped.  The workspace lives until kc_graph_destroy.
 * Errors: KC_ERR_INVALID (count < 1), KC_ERR_NOMEM (the budget of
 * KC_OPT_MEM_BUDGET, or 80% of free device memory, cannot hold one sample),
 * KC_ERR_DEVICE.
 */
kc_status kc_reserve(kc_graph *g, int32_t count, void *hip_stream);

/*
 * Free g's device workspace (the per-sample sampler and numbering state of
 * the samples in flight) and its internal per-sample result buffers now; the
 * next call that needs them allocates them again.  The graph arrays and the
 * resident sample set stay.  For callers that hand the memory to other work
 * between estimates (a serving loop after an update, a captured batch).
 * Errors: KC_ERR_INVALID (NULL graph), KC_ERR_DEVICE.
 */
kc_status kc_trim(kc_graph *g, void *hip_stream);

/*
 * Draw the uniform spanning trees of samples first_sample ..
 * first_sample+count-1 with Wilson's algorithm (section 2.2), each
 * (sample s, vertex v, k-th draw at v) taking neighbour slot
 * floor(x * deg(v) / 2^64) of v's row, where x = o0 | o1 << 32 are the first
 * two words of Philox4x32-10 (Salmon et al., SC'11) with counter
 * (k, v, s_lo, s_hi) and key (seed_lo, seed_hi).  Many walkers cooperate on
 * one sample by cycle popping, so the tree and the per-vertex draw counts are
 * the unique cycle-popping outcome of these arrows.
 *   parents_out   : DEVICE pointer, count*n int32, row i = sample first+i,
 *                   parents_out[i*n + v] = parent of v in the tree (root: -1)
 *   popcounts_out : DEVICE pointer or NULL, count*n uint32, number of draws
 *                   made at v (0 at the root)
 *   steps_out     : DEVICE pointer or NULL, count int64, total draws per sample
 * Errors: KC_ERR_INVALID (count < 0, NULL parents_out with count > 0),
 * KC_ERR_LIMIT, KC_ERR_NOMEM, KC_ERR_DEVICE.
 */
kc_status kc_sample_trees(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                          int32_t *parents_out, uint32_t *popcounts_out, int64_t *steps_out,
                          void *hip_stream);

/* Result of an estimate (host struct). */
typedef struct {
    double kappa;        /* (double)(sum f) / (2m * count): one rounding of the exact sum,
                            one division (Algorithm 1, last line; Theorem 3.3) */
    double std_error;    /* sample standard deviation of f/2m over sqrt(count) */
    uint64_t sum_f_lo;   /* exact sum of f as a two's-complement 128-bit integer */
    int64_t sum_f_hi;
    uint64_t sum_f2_lo;  /* exact sum of f^2 (unsigned 128-bit) */
    uint64_t sum_f2_hi;
    int64_t count;
    int64_t total_steps; /* Wilson draws over all samples */
    int64_t sampler_iterations; /* lock-step sampler rounds over all samples; total_steps divided
                                   by this is the mean number of walkers drawing per round */
} kc_result;

/*
 * Sample trees first_sample .. first_sample+count-1 (as kc_sample_trees)
 * and evaluate f(tau) for each on the device (Theorems 3.3/3.4), then reduce
 * exactly.  f is an exact int64 per tree.
 *   result : HOST pointer (required)
 *   f_out  : DEVICE pointer or NULL, count int64 per-sample f
 *   steps_out : DEVICE pointer or NULL, count int64 draws per sample
 * Errors: as kc_sample_trees; KC_ERR_INVALID for count < 1.
 */
kc_status kc_estimate(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                      kc_result *result, int64_t *f_out, int64_t *steps_out, void *hip_stream);

/*
 * Pool results of the same graph over disjoint sample ranges (for example the
 * successive batches of a long run) into one estimate of Theorem 3.3 over all
 * their samples: the exact sums and counts add, and kappa and std_error are
 * recomputed from the pooled sums exactly as kc_estimate computes them.
 *   parts : HOST pointer, k results of kc_estimate (or of other calls that
 *           fill kc_result) on this graph; out : HOST pointer
 * Errors: KC_ERR_INVALID (NULL argument, k < 1, a part with count < 1).
 */
kc_status kc_combine_results(const kc_graph *g, const kc_result *parts, int32_t k, kc_result *out);

/*
 * kc_estimate for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results as kc_estimate (bit for bit); it allocates
 * nothing (no hipMalloc, hipFree or allocating library call).  Its workspace
 * is one static device array of 256 MiB per device, held until the process
 * ends: the per-sample results first (24 bytes per sample, 16 when f_out is
 * given), then as many samples in flight as fit (kc_graph_info.sample_bytes
 * each, at most the slots option or the kernel's resident workgroups).
 * Every call on a device shares that array and leaves the last call's
 * contents in it, so calls that overlap on one device race: callers
 * serialise them.  The graph must have been created (kc_graph_create
 * allocates its arrays); this call then allocates nothing.
 *   result : HOST pointer (required); f_out : DEVICE pointer or NULL
 * Errors: KC_ERR_INVALID (count < 1, NULL graph or result), KC_ERR_NOMEM (the
 * per-sample results, or one sample in flight, do not fit the static
 * workspace), KC_ERR_LIMIT, KC_ERR_DEVICE.
 */
kc_status kc_estimate_static(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                             kc_result *result, int64_t *f_out, void *hip_stream);

/*
 * Batches (section 5, Exp-VI parallelises across samples; here the samples of
 * several graphs of any sizes share one persistent launch).  A batch holds up
 * to 8 graphs, one job each: launch number L (from 0) of the batch estimates
 * samples firsts[j] + L*counts[j] .. firsts[j] + (L+1)*counts[j] - 1 of graph
 * j, each tree bit-identical to kc_estimate's for the same (seed, s).  The
 * launch sequence (status reset, the persistent kernel over every job, the
 * exact sums of each job, the launch counter) is captured once as a HIP graph
 * at creation and replayed by kc_batch_launch with no host round trip: the
 * status and sums stay on the device until kc_batch_results reads them.
 * Launch options (step limit, walkers, traversal) are each
 * graph's; the chain-table size, samples in flight and memory budget are the
 * first graph's; lean looks (KC_OPT_LEAN_LOOKS) are taken only when every
 * graph of the batch takes them (results do not depend on either).  The batch owns its workspace (slots sized for the largest
 * graph) and copies of the graphs' device array pointers: the graphs must
 * outlive the batch and must not be updated (kc_apply_updates, kc_set_tau0)
 * while it exists.
 */
typedef struct kc_batch kc_batch;

/*
 *   graphs : HOST array of k graph handles (1 <= k <= 8)
 *   seeds, firsts, counts : HOST arrays of k entries (counts >= 1, firsts >= 0,
 *            sum of counts < 2^31)
 *   out    : receives the batch
 * Errors: KC_ERR_INVALID, KC_ERR_NOMEM (one sample of the largest graph does not
 * fit the budget), KC_ERR_DEVICE (capture failed).
 */
kc_status kc_batch_create(kc_graph *const *graphs, int32_t k, const uint64_t *seeds, const int64_t *firsts,
                          const int32_t *counts, void *hip_stream, kc_batch **out);

/* Enqueue the next launch of the batch on hip_stream (a graph replay); returns
 * at once.  Launches on one batch must be ordered (one stream). */
kc_status kc_batch_launch(kc_batch *b, void *hip_stream);

/* Wait for hip_stream, then read the last launch's status and results:
 * results HOST [k] (as kc_estimate's for each job), launches HOST or NULL
 * (launches completed so far).  Errors: the last launch's KC_ERR_LIMIT or
 * KC_ERR_DEVICE (results then unspecified). */
kc_status kc_batch_results(kc_batch *b, kc_result *results, int64_t *launches, void *hip_stream);

/* Copy job j's per-sample f of the last launch (counts[j] int64) to the DEVICE
 * pointer f_out. */
kc_status kc_batch_f(const kc_batch *b, int32_t j, int64_t *f_out, void *hip_stream);

/* Free the batch (its captured graph and workspace).  NULL is accepted. */
kc_status kc_batch_destroy(kc_batch *b);

/* Launch options chosen by kc_autotune. */
typedef struct {
    int32_t chains, slots, walkers, traversal; /* as KC_OPT_* values */
    int32_t from_cache;   /* 1 if read from the cache file, 0 if measured now */
    int32_t trials;       /* trial estimates run */
    double samples_per_s; /* rate of the chosen options in their trial (0 from the cache) */
    double start_samples_per_s; /* rate of the options the graph had before (0 from the cache) */
} kc_tune_result;

/*
 * Choose g's launch options for estimates of `count` samples by timing short
 * trial estimates (one wave of samples in flight, at least 64, on sample ids
 * from 2^40 upward): starting from the current options, one option at a
 * time (traversal for tau0 depth <= 64, chain-table size,
 * 3/4 and 1/2 of the samples in flight, walkers 32/64), a change kept only for
 * a gain above 2%.  The choice is applied to g (kc_set_option) and appended to
 * cache_path (HOST string or NULL: no cache) as one JSON line keyed by device
 * architecture, n, 2m, max degree, tau0 depth and count; a later call with the
 * same key applies the cached choice without trials.  No option changes any
 * result (trees, f and estimates are bit-identical).
 *   out : HOST pointer
 * Errors: those of kc_estimate (the options are then put back).
 */
kc_status kc_autotune(kc_graph *g, int32_t count, const char *cache_path, kc_tune_result *out, void *hip_stream);

/*
 * Evaluate f for caller-supplied rooted spanning trees (no sampling).
 *   parents : DEVICE pointer, count*n int32 parent arrays rooted at the
 *             graph's root (root -> -1; the root's entry is not read).
 *             Every edge (v, parent[v]) should be a graph edge.
 *   f_out   : DEVICE pointer, count int64
 * The kernels check each array: a parent out of range or equal to its vertex,
 * or parents that do not form one tree rooted at r (a cycle, a vertex that
 * does not reach r), give KC_ERR_INVALID.  Whether each (v, parent[v]) is an
 * edge of the graph is not checked; f of such an array is that of the tree
 * it describes, on the graph's degrees.
 */
kc_status kc_evaluate_trees(kc_graph *g, const int32_t *parents, int32_t count, int64_t *f_out,
                            void *hip_stream);

/*
 * Samples finished so far by the sampling call running (or last run) on g:
 * each workgroup of the persistent kernel publishes its count to pinned host
 * memory after every sample.  Unlike every other call, this one may be made
 * from another host thread while kc_sample_trees / kc_estimate /
 * kc_evaluate_trees is running on the same graph; it reads host memory only
 * and never blocks on the device.
 *   samples_done : HOST pointer, receives the count
 * Errors: KC_ERR_INVALID (NULL argument).
 */
kc_status kc_progress(const kc_graph *g, int64_t *samples_done);

/*
 * Resident sample set (section 4: the sample set S kept between updates).
 *
 * kc_samples_init draws the trees of samples 0 .. count-1 (as
 * kc_sample_trees, with `seed`) and keeps their parent arrays and f values
 * on the device with the graph.  Replaces any earlier set; on an error no
 * set is resident afterwards.
 * Errors: as kc_sample_trees; KC_ERR_INVALID for count < 1.
 */
kc_status kc_samples_init(kc_graph *g, uint64_t seed, int32_t count, void *hip_stream);

/* kc_estimate's result over the resident trees on the current graph
 * (Theorem 3.3 with omega = the set's size).  result: HOST pointer.
 * Under KC_MAINT_IMPROVED, kappa is the weighted estimate sum_t w_t f_t / 2m
 * (Algorithm 3, weights summing to one, added in slot order) and std_error
 * is sqrt(sum_t w_t^2 (f_t / 2m - kappa)^2); the exact sums stay unweighted.
 * Errors: KC_ERR_INVALID if no set was initialised. */
kc_status kc_samples_query(kc_graph *g, kc_result *result, void *hip_stream);

/* The resident trees' weights (HOST pointer, the set's size in doubles):
 * 1/count after kc_samples_init, changed only by improved maintenance.
 * Errors: KC_ERR_INVALID (NULL argument, no set). */
kc_status kc_samples_weights(const kc_graph *g, double *w_out);

/* Copy the resident set out: parents_out DEVICE [count*n] int32, f_out
 * DEVICE [count] int64, ids_out HOST [count] int64 (the sample index each
 * tree was drawn with); any may be NULL.  count is the set's size.  If the
 * last update could not recompute f on the device, f is recomputed first
 * (kc_samples_query does the same), and its failure is returned. */
kc_status kc_samples_get(kc_graph *g, int32_t *parents_out, int64_t *f_out, int64_t *ids_out,
                         void *hip_stream);

/*
 * Apply a list of edge updates (section 4.1, Algorithm 2: basic sample
 * maintenance), in order.  A run of consecutive deletions is applied at
 * once; each insertion is applied on its own.  tau0 and every per-graph array
 * are rebuilt on the new graph with the same root, and f is recomputed for
 * every resident tree, since degrees, 2m and tau0 change.
 *   Deletion of (u, v), an edge of the graph (distinct within a run): the
 *     graph after the run must stay connected.  Resident trees that contain
 *     a deleted edge are replaced by fresh uniform spanning trees of the new
 *     graph (the set's seed, the next unused sample indices, in slot order);
 *     the others are uniform on it already (Theorem 4.2).
 *   Insertion of (u, v), not an edge of the graph: R(u, v) on the graph
 *     before it is estimated from the resident trees (the signed count of
 *     the edges of a fixed breadth-first u -> v path that each tree's own
 *     u -> v path uses; its mean is R(u, v)).  Each resident tree is then
 *     replaced independently with probability R / (1 + R), the probability
 *     that a uniform spanning tree of the new graph uses the new edge
 *     (Theorem 4.1), by the draw (x >> 11) * 2^-53 with x the first two words
 *     of Philox4x32-10, key (seed_lo, seed_hi), counter (slot, number of
 *     insertions applied to the set so far, 2^32-1, 2^32-1).  A replacement
 *     is a uniform spanning tree through the new edge: Wilson's algorithm with
 *     u and v in the tree from the start (next unused sample index), the edge
 *     v -> u added, and the path from the root re-oriented toward it.
 *   u, v, is_insert : HOST pointers, count entries (is_insert NULL: all deletions)
 *   resampled       : HOST pointer or NULL, receives how many trees were replaced
 *
 * Under KC_MAINT_IMPROVED (section 4.2, Algorithm 3) every edge is applied on
 * its own, in order, and trees are transformed instead of redrawn; Philox
 * with key (seed_lo, seed_hi) and counter (slot, j, 2^32-2, 2^32-1) picks an
 * edge among d candidates as floor(x d / 2^64), j counting the edges applied
 * to the set so far:
 *   Insertion of e = (u, v): R on the graph before it is estimated from the
 *     weighted trees (sum_t w_t times the signed path count above); ceil(R' n_S)
 *     trees (R' = R / (1 + R), n_S the set's size) are chosen, those with the
 *     smallest replacement draws of the basic case.  Each goes through
 *     link-cut: e is added and one of the d edges of the tree path between u
 *     and v removed (counted from u upward, then from v upward).  Its weight is
 *     multiplied by d / d', d' being the number of edges of the old graph that
 *     join the two parts of the new tree minus e (Theorem 4.4).  The chosen
 *     trees' weights are then scaled to sum to R', the others' to 1 - R'.
 *   Deletion of e: each tree through e goes through cut-link: e is removed and
 *     one of the d edges of the new graph that join the two parts added (edges
 *     {x, y}, x < y, by x, then in row order).  Its weight is multiplied by
 *     d / d', d' being the length of the new tree's path between u and v
 *     (Theorem 4.5), and these trees' weights are scaled back to their total
 *     before the update.
 *   Sample indices do not change; resampled receives the trees transformed.
 * Errors: KC_ERR_INVALID (a deletion that is not an edge, a duplicate within a
 * run, an insertion of an existing edge, a bad vertex), KC_ERR_DISCONNECTED
 * (a deletion run would disconnect the graph), KC_ERR_OVERFLOW (2m would
 * reach 2^31), and those of kc_sample_trees.  Updates before the failing one
 * stay applied; the failing one changes nothing, also when it fails on the
 * device after the graph was switched (the previous graph and trees are put
 * back).  f of the resident trees is recomputed once at the end of the call;
 * if that recomputation fails (for example KC_ERR_NOMEM when the graph grew
 * past KC_OPT_MEM_BUDGET), the call returns its error with the updates in
 * place, and f stays marked stale: kc_samples_query and kc_samples_get
 * recompute it first and return the failure again while it persists, so no
 * query ever reduces f values of an earlier graph.  A run of deletions
 * counts as one update under KC_MAINT_BASIC and as one update per edge under
 * KC_MAINT_IMPROVED.
 */
kc_status kc_apply_updates(kc_graph *g, const int32_t *u, const int32_t *v, const uint8_t *is_insert,
                           int32_t count, int32_t *resampled, void *hip_stream);

/* Static description of a status code. */
const char *kc_status_string(kc_status s);

/* Detail message of the calling thread's last failing call ("" if none). */
const char *kc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
