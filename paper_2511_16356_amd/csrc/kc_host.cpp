// kc_host.cpp -- C ABI (include/kc.h): validation, graph preparation,
// device workspace and launches.  Graph preparation (root, tau0 by its rule,
// tau0 preorder) runs once per graph version on the host; everything per
// sample runs in the kernels of kc_device.hip.  The sample maintenance of
// section 4 keeps its bookkeeping here (which trees to replace or transform,
// the weights of Algorithm 3, the switch to the updated graph and its undo on
// failure); the per-tree work runs on the device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "kc_host.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

kc_status kc_host::fail(kc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

using namespace kc_host;

namespace {

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

// A temporary device buffer freed when it goes out of scope (also on the
// early returns of HIP_TRY).
template <typename T>
struct DevTmp {
    T *p = nullptr;
    hipStream_t s = nullptr;
    DevTmp() = default;
    DevTmp(const DevTmp &) = delete;
    DevTmp &operator=(const DevTmp &) = delete;
    ~DevTmp() {
        if (p) (void)hipFreeAsync(p, s);
    }
    // stream-ordered: neither the allocation nor the free waits for work on other
    // streams (a plain hipFree synchronises the whole device)
    hipError_t alloc(size_t count, hipStream_t stream) {
        s = stream;
        return hipMallocAsync(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T), stream);
    }
};

// Runs body(lo, hi) over [0, n) in contiguous chunks on up to 16 host threads
// and returns the smallest index any chunk reported (body returns its first
// failing index, or -1), so errors are reported as a serial scan would.
template <typename F>
int64_t parallel_first(int64_t n, F body) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (n < (1 << 16)) nt = 1;
    std::vector<int64_t> first(nt, -1);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        if (nt == 1) first[t] = body(lo, hi);
        else th.emplace_back([&, t, lo, hi] { first[t] = body(lo, hi); });
    }
    for (auto &x : th) x.join();
    for (int64_t f : first)
        if (f >= 0) return f;
    return -1;
}

}  // namespace

namespace {

void free_workspace(kc_graph *g) {
    dev_free(g->d_state); dev_free(g->d_queue); dev_free(g->d_cstart); dev_free(g->d_rec);
    dev_free(g->d_fen);
    g->d_state = nullptr; g->d_queue = nullptr; g->d_cstart = nullptr;
    g->d_rec = nullptr; g->d_fen = nullptr;
    g->ws_slots = 0; g->ws_asked = 0; g->ws_trav = g->ws_fen = false;
}

void free_graph_arrays(kc_graph *g);

void free_all(kc_graph *g) {
    free_workspace(g);
    free_graph_arrays(g);
    dev_free(g->d_res_par); dev_free(g->d_res_f); dev_free(g->d_res_f_alt);
    g->d_res_par = nullptr; g->d_res_f = nullptr; g->d_res_f_alt = nullptr; g->res_count = 0;
    dev_free(g->d_f); dev_free(g->d_steps); dev_free(g->d_iters); dev_free(g->d_ctl); dev_free(g->d_red);
    if (g->h_progress) (void)hipHostFree(g->h_progress);
    g->h_progress = nullptr;
    g->d_progress = nullptr;
    g->progress_len = 0;
}

// Walk start orders.  Wilson's algorithm may start its walks in any order
// and the cycle-popping outcome is the same; the order only changes how often
// concurrent walks run into each other.  Walks started at scattered random
// vertices collide far less than walks started in BFS order around the root.
std::vector<int32_t> start_order_of(const std::vector<int32_t> &bfs, int kind) {
    std::vector<int32_t> ord = bfs;
    if (kind == 1) std::reverse(ord.begin(), ord.end());
    if (kind == 2) {
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (size_t i = ord.size(); i > 1; --i) {  // Fisher-Yates driven by splitmix64
            x += 0x9E3779B97F4A7C15ull;
            uint64_t z = x;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            std::swap(ord[i - 1], ord[(size_t)(z % i)]);
        }
    }
    return ord;
}

}  // namespace

int64_t kc_host::slot_bytes(const kc_graph *g, bool trav, bool fen) {
    // sampler state (reused by the numbering's ord and grp), tasks and chain starts
    int64_t b = kc::state_bytes(g->n) + 20 * (int64_t)kc::sampler_chains();
    if (trav) b += 16 * g->n;  // rec
    if (fen) b += 8 * (g->two_m + 2);
    return b;
}

namespace {

// Make sure at least `want` slots of workspace exist; returns the usable count.
kc_status ensure_workspace(kc_graph *g, int want, bool trav, bool fen, hipStream_t stream, int *got) {
    if (want < 1) want = 1;
    // the sweep's per-slot stride is 2m + 2: a graph that gained edges needs a new buffer
    const bool fen_small = fen && g->ws_fen && g->ws_fen_len < g->two_m + 2;
    // a workspace asked for at least `want` slots is kept, also when the budget held fewer
    if ((g->ws_slots >= want || g->ws_asked >= want) && (!trav || g->ws_trav) && (!fen || g->ws_fen) &&
        !fen_small) {
        *got = std::min(want, g->ws_slots);
        return KC_OK;
    }
    trav = trav || g->ws_trav;
    fen = fen || g->ws_fen;
    want = std::max(want, g->ws_slots);
    free_workspace(g);
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const int64_t budget = workspace_budget(g, free_b);
    const int64_t per = slot_bytes(g, trav, fen);
    int64_t fit = budget / per;
    if (fit < 1) return fail(KC_ERR_NOMEM, "one sample needs %lld bytes of workspace, budget %lld",
                             (long long)per, (long long)budget);
    int slots = (int)std::min<int64_t>(want, fit);
    const size_t n = (size_t)g->n;
    HIP_TRY(dev_alloc(&g->d_state, (size_t)slots * (size_t)kc::state_bytes(g->n)));
    HIP_TRY(dev_alloc(&g->d_queue, (size_t)slots * (size_t)kc::sampler_chains()));
    HIP_TRY(dev_alloc(&g->d_cstart, (size_t)slots * (size_t)kc::sampler_chains()));
    if (trav) HIP_TRY(dev_alloc(&g->d_rec, (size_t)slots * n));
    if (fen) {
        const int64_t len = (int64_t)slots * (g->two_m + 2);
        HIP_TRY(dev_alloc(&g->d_fen, (size_t)len));
        HIP_TRY(kc::launch_zero_i64(g->d_fen, len, stream));
    }
    g->ws_slots = slots;
    g->ws_asked = want;
    g->ws_trav = trav;
    g->ws_fen = fen;
    g->ws_fen_len = fen ? g->two_m + 2 : 0;
    *got = slots;
    return KC_OK;
}

kc_status ensure_fbuf(kc_graph *g, int64_t count) {
    if (g->fbuf_len >= count) return KC_OK;
    dev_free(g->d_f);
    dev_free(g->d_steps);
    dev_free(g->d_iters);
    g->d_f = g->d_steps = g->d_iters = nullptr;
    g->fbuf_len = 0;
    HIP_TRY(dev_alloc(&g->d_f, (size_t)count));
    HIP_TRY(dev_alloc(&g->d_steps, (size_t)count));
    HIP_TRY(dev_alloc(&g->d_iters, (size_t)count));
    g->fbuf_len = count;
    return KC_OK;
}

}  // namespace

// One slot per resident single-wave workgroup of the persistent kernel.
int kc_host::default_slots(const kc_graph *g, bool batch) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    per_cu = batch ? kc::batch_blocks_per_cu(g->chains) : kc::persistent_blocks_per_cu(g->chains);
    if (cus <= 0 || per_cu <= 0) return 1024;
    return cus * per_cu;
}

// Workspace bytes a launch may allocate: the graph's budget option, else 80%
// of the device memory free before the allocation.
int64_t kc_host::workspace_budget(const kc_graph *g, size_t free_b) {
    return g->mem_budget > 0 ? g->mem_budget : (int64_t)(0.8 * (double)free_b);
}


// Samples in flight for a launch of `count` samples on up to `slots` slots:
// as many as give every wave of samples the same size (ceil(count / waves)
// for the fewest waves), so that a launch does not end with a wave of a few
// samples running nearly alone.
int kc_host::balanced_slots(int slots, int64_t count) {
    if (slots < 1 || count <= slots) return slots;
    const int64_t waves = (count + slots - 1) / slots;
    return (int)((count + waves - 1) / waves);
}

// The graph's device arrays as the kernels see them.
kc::GraphDev kc_host::graph_dev(const kc_graph *g) {
    kc::GraphDev gd;
    gd.n = (int32_t)g->n;
    gd.root = g->root;
    gd.two_m = g->two_m;
    gd.off = g->d_off;
    gd.adj = g->d_adj;
    gd.p0 = g->d_p0;
    gd.order = g->d_order;
    gd.pre0 = g->d_pre0;
    gd.out0 = g->d_out0;
    gd.eoff = g->d_eoff;
    gd.elist = g->d_elist;
    gd.vrec = g->d_vrec;
    gd.anc0 = g->d_anc0;
    gd.anc_depth = g->anc_depth;
    return gd;
}


// The options of g that every launch carries.
void kc_host::fill_run_options(const kc_graph *g, kc::RunParams &rp) {
    rp.walkers = g->walkers;
    rp.traversal = g->traversal;
    // lean looks pay where walks are short, so that most looks at a walk's next
    // vertex meet the tree: by default when the mean degree is at least 8
    rp.lean = g->lean_opt == 2 || (g->lean_opt == 0 && g->two_m >= 8 * g->n);
    rp.iter_cap = g->step_limit > 0 ? g->step_limit : 1024 * g->n + (1 << 22);
    rp.ctl = g->d_ctl;
}


// Launch the persistent kernel on a prepared workspace and check the status
// its workgroups report.
kc_status kc_host::launch_checked(kc_graph *g, const kc::SlotDev &sd, const kc::RunParams &rp, int slots,
                         hipStream_t stream) {
    HIP_TRY(kc::launch_reset_ctl(g->d_ctl, stream));
    HIP_TRY(kc::launch_persistent(graph_dev(g), sd, rp, g->chains, slots, stream));
    int32_t ctl[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(ctl, g->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (ctl[1] != 0) {
        if (ctl[1] == kc::DEV_LIMIT)
            return fail(KC_ERR_LIMIT, "sample %lld exceeded the step limit",
                        (long long)(rp.first + ctl[2]));
        if (ctl[1] == kc::DEV_BADTREE)
            return fail(KC_ERR_INVALID, "parents of tree %d do not form a spanning tree rooted at %d",
                        ctl[2], g->root);
        return fail(KC_ERR_DEVICE, "sampler protocol violation (code %d) in sample %lld", ctl[1],
                    (long long)(rp.first + ctl[2]));
    }
    return KC_OK;
}

namespace {

// Launch the persistent kernel over `count` samples on the graph's own
// workspace (allocated or grown here) and check its status.
kc_status run_persistent(kc_graph *g, kc::RunParams rp, hipStream_t stream) {
    const bool trav = rp.mode != kc::RUN_SAMPLE;
    const bool fen = trav && g->traversal == KC_TRAV_SWEEP;
    int want = g->slots_opt > 0 ? g->slots_opt : default_slots(g);
    want = std::min(want, rp.count);
    int slots = 0;
    kc_status st = ensure_workspace(g, want, trav, fen, stream, &slots);
    if (st != KC_OK) return st;
    slots = balanced_slots(slots, rp.count);
    kc::SlotDev sd;
    sd.state = g->d_state;
    sd.queue = g->d_queue;
    sd.cstart = g->d_cstart;
    sd.chains = kc::sampler_chains();
    sd.rec = trav ? g->d_rec : nullptr;
    sd.stride = g->n;
    sd.fen = fen ? g->d_fen : nullptr;
    sd.fen_len = fen ? g->two_m + 2 : 0;
    fill_run_options(g, rp);
    if (g->progress_len < slots) {
        if (g->h_progress) (void)hipHostFree(g->h_progress);
        g->h_progress = nullptr;
        g->d_progress = nullptr;
        g->progress_len = 0;
        HIP_TRY(hipHostMalloc((void **)&g->h_progress, sizeof(int64_t) * (size_t)slots,
                              hipHostMallocMapped | hipHostMallocCoherent));
        HIP_TRY(hipHostGetDevicePointer((void **)&g->d_progress, g->h_progress, 0));
        g->progress_len = slots;
    }
    HIP_TRY(hipStreamSynchronize(stream));  // no earlier launch still writes the counters
    for (int i = 0; i < g->progress_len; ++i) __atomic_store_n(&g->h_progress[i], (int64_t)0, __ATOMIC_RELAXED);
    rp.progress = g->d_progress;
    return launch_checked(g, sd, rp, slots, stream);
}

// Philox4x32-10 (Salmon et al., SC'11) on the host: ten rounds of two 32x32
// products with the Weyl key increments.
void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * x0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        x0 = y0; x1 = (uint32_t)b; x2 = y2; x3 = (uint32_t)a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// The replacement draw of resident tree `slot` at insertion number `serial`:
// counter (slot, serial, 2^32-1, 2^32-1), which no tree sample uses; the first
// two output words as a 64-bit x, uniform = (x >> 11) * 2^-53 in [0, 1).
double update_uniform(uint64_t seed, uint32_t slot, uint32_t serial) {
    const uint32_t ctr[4] = {slot, serial, 0xFFFFFFFFu, 0xFFFFFFFFu};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    philox_host(ctr, key, o);
    const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    return (double)(x >> 11) * 0x1.0p-53;
}

// A fixed u -> v path: breadth-first search from u (rows ascending), each
// vertex reached from the first vertex that reaches it.
std::vector<int32_t> reference_path(const std::vector<int64_t> &off, const std::vector<int32_t> &adj,
                                    int32_t u, int32_t v) {
    const int64_t n = (int64_t)off.size() - 1;
    std::vector<int32_t> pred((size_t)n, -1), q;
    pred[(size_t)u] = u;
    q.push_back(u);
    for (size_t h = 0; h < q.size() && pred[(size_t)v] < 0; ++h) {
        const int32_t x = q[h];
        for (int64_t e = off[(size_t)x]; e < off[(size_t)x + 1]; ++e) {
            const int32_t y = adj[(size_t)e];
            if (pred[(size_t)y] < 0) { pred[(size_t)y] = x; q.push_back(y); }
        }
    }
    std::vector<int32_t> path;
    if (pred[(size_t)v] < 0) return path;
    for (int32_t x = v;; x = pred[(size_t)x]) {
        path.push_back(x);
        if (x == u) break;
    }
    std::reverse(path.begin(), path.end());
    return path;
}

// (Re)build every per-graph array from the host CSR in g->h_off / g->h_adj:
// root (highest degree, smallest index, unless given), tau0 (by `tau0_kind`:
// BFS with parent = smallest-index neighbour one level up, depth-first from the
// root with rows in ascending order, or the caller's tree in `given`), tau0
// preorder and subtree ends, the per-block open-subtree lists, the walk start
// order and the per-vertex graph records; then replace the device copies.  On
// failure the graph is unchanged only if nothing was uploaded yet (callers
// validate first).
kc_status prepare_graph(const std::vector<int64_t> &off, const std::vector<int32_t> &adj, int32_t root,
                        int tau0_kind, const std::vector<int32_t> *given, PreparedGraph *pg) {
    const int64_t n = (int64_t)off.size() - 1;
    const int64_t nnz = off[(size_t)n];
    const int32_t *indices = adj.data();
    if (root < 0) {
        int64_t best = -1;
        for (int64_t v = 0; v < n; ++v) {
            const int64_t d = off[(size_t)v + 1] - off[(size_t)v];
            if (d > best) { best = d; root = (int32_t)v; }
        }
    }
    if (root < 0 || root >= n) return fail(KC_ERR_INVALID, "root %d out of range", root);
    pg->root = root;
    // BFS from the root; the queue order is the walk start order
    std::vector<int32_t> dist((size_t)n, -1);
    std::vector<int32_t> &order = pg->order;
    order.clear();
    order.reserve((size_t)n);
    dist[(size_t)root] = 0;
    order.push_back(root);
    for (size_t h = 0; h < order.size(); ++h) {
        const int32_t x = order[h];
        for (int64_t e = off[(size_t)x]; e < off[(size_t)x + 1]; ++e) {
            const int32_t y = indices[e];
            if (dist[(size_t)y] < 0) {
                dist[(size_t)y] = dist[(size_t)x] + 1;
                order.push_back(y);
            }
        }
    }
    if ((int64_t)order.size() != n)
        return fail(KC_ERR_DISCONNECTED, "only %zu of %lld vertices reachable from the root", order.size(), (long long)n);
    std::vector<int32_t> &p0 = pg->p0;
    p0.assign((size_t)n, -1);
    int32_t depth0 = 0;
    if (tau0_kind == KC_TAU0_BFS) {
        // parent = smallest-index neighbour one level up
        for (int64_t v = 0; v < n; ++v) {
            depth0 = std::max(depth0, dist[(size_t)v]);
            if (v == root) continue;
            for (int64_t e = off[(size_t)v]; e < off[(size_t)v + 1]; ++e) {
                const int32_t u = indices[e];
                if (dist[(size_t)u] == dist[(size_t)v] - 1) { p0[(size_t)v] = u; break; }  // rows ascending
            }
        }
    } else if (tau0_kind == KC_TAU0_DFS) {
        // depth-first search from the root, each row scanned in ascending order;
        // a vertex's parent is the vertex it was discovered from
        std::vector<int64_t> pos((size_t)n);
        std::vector<int32_t> depth((size_t)n, -1), stack;
        stack.push_back(root);
        depth[(size_t)root] = 0;
        pos[(size_t)root] = off[(size_t)root];
        while (!stack.empty()) {
            const int32_t x = stack.back();
            if (pos[(size_t)x] == off[(size_t)x + 1]) { stack.pop_back(); continue; }
            const int32_t y = indices[pos[(size_t)x]++];
            if (depth[(size_t)y] >= 0) continue;
            depth[(size_t)y] = depth[(size_t)x] + 1;
            depth0 = std::max(depth0, depth[(size_t)y]);
            p0[(size_t)y] = x;
            pos[(size_t)y] = off[(size_t)y];
            stack.push_back(y);
        }
    } else if (tau0_kind == KC_TAU0_GIVEN && given && (int64_t)given->size() == n) {
        // the caller's tree: parent[root] = -1, every (v, parent[v]) an edge, no cycle
        const std::vector<int32_t> &t = *given;
        if (t[(size_t)root] != -1) return fail(KC_ERR_INVALID, "tau0: parent of the root %d must be -1", root);
        for (int64_t v = 0; v < n; ++v) {
            if (v == root) continue;
            const int32_t u = t[(size_t)v];
            if (u < 0 || u >= n) return fail(KC_ERR_INVALID, "tau0: parent %d of %lld out of range", u, (long long)v);
            if (!std::binary_search(indices + off[(size_t)v], indices + off[(size_t)v + 1], u))
                return fail(KC_ERR_INVALID, "tau0: (%lld,%d) is not an edge of the graph", (long long)v, u);
        }
        std::vector<int32_t> depth((size_t)n, -1), chain;
        depth[(size_t)root] = 0;
        for (int64_t v = 0; v < n; ++v) {
            int32_t x = (int32_t)v;
            chain.clear();
            while (depth[(size_t)x] < 0) {  // at most n steps: a longer chain repeats a vertex
                if ((int64_t)chain.size() >= n)
                    return fail(KC_ERR_INVALID, "tau0: the parent array has a cycle through %lld", (long long)v);
                chain.push_back(x);
                x = t[(size_t)x];
            }
            for (size_t i = chain.size(); i-- > 0;) depth[(size_t)chain[i]] = depth[(size_t)x] + (int32_t)(chain.size() - i);
        }
        p0 = t;
        for (int64_t v = 0; v < n; ++v) depth0 = std::max(depth0, depth[(size_t)v]);
    } else {
        return fail(KC_ERR_INVALID, "unknown tau0 rule %d (or a given tree of the wrong size)", tau0_kind);
    }
    pg->depth0 = depth0;
    const unsigned __int128 bound = (unsigned __int128)nnz * (unsigned __int128)nnz * (unsigned __int128)depth0;
    if (bound >= ((unsigned __int128)1 << 63))
        return fail(KC_ERR_OVERFLOW, "4 m^2 depth0 = (2m)^2 * %d exceeds 2^63", depth0);
    // tau0 preorder, children in ascending order
    std::vector<int64_t> cst((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v) if (v != root) cst[(size_t)p0[(size_t)v] + 1]++;
    for (int64_t v = 0; v < n; ++v) cst[(size_t)v + 1] += cst[(size_t)v];
    std::vector<int32_t> clist((size_t)n);
    {
        std::vector<int64_t> fill(cst.begin(), cst.end() - 1);
        for (int64_t v = 0; v < n; ++v) if (v != root) clist[(size_t)fill[(size_t)p0[(size_t)v]]++] = (int32_t)v;
    }
    std::vector<int32_t> in0((size_t)n);
    std::vector<int32_t> &pre0 = pg->pre0, &out0 = pg->out0;
    pre0.assign((size_t)n, 0);
    out0.assign((size_t)n, 0);
    {
        std::vector<int32_t> stack;
        std::vector<int64_t> next((size_t)n);
        int32_t t = 0;
        stack.push_back(root);
        next[(size_t)root] = cst[(size_t)root];
        pre0[(size_t)t] = root;
        in0[(size_t)root] = t++;
        while (!stack.empty()) {
            const int32_t x = stack.back();
            if (next[(size_t)x] < cst[(size_t)x + 1]) {
                const int32_t c = clist[(size_t)next[(size_t)x]++];
                next[(size_t)c] = cst[(size_t)c];
                pre0[(size_t)t] = c;
                in0[(size_t)c] = t++;
                stack.push_back(c);
            } else {
                out0[(size_t)x] = t - 1;
                stack.pop_back();
            }
        }
    }
    // per 64-position block: tau0 vertices whose subtree opened before the block and closes in it
    const int32_t nblk = (int32_t)((n + 63) / 64);
    pg->nblk = nblk;
    std::vector<int32_t> &eoff = pg->eoff, &elist = pg->elist;
    eoff.assign((size_t)nblk + 1, 0);
    for (int64_t x = 0; x < n; ++x) {
        const int32_t be = out0[(size_t)x] / 64;
        if (in0[(size_t)x] < be * 64) eoff[(size_t)be + 1]++;
    }
    for (int32_t b = 0; b < nblk; ++b) eoff[(size_t)b + 1] += eoff[(size_t)b];
    elist.assign((size_t)eoff[(size_t)nblk], 0);
    {
        std::vector<int32_t> fill(eoff.begin(), eoff.end() - 1);
        for (int64_t x = 0; x < n; ++x) {
            const int32_t be = out0[(size_t)x] / 64;
            if (in0[(size_t)x] < be * 64) elist[(size_t)fill[(size_t)be]++] = (int32_t)x;
        }
    }
    // shallow tau0 (depth <= 8): every vertex's tau0 ancestors, level-major and padded to 4 or
    // 8 levels with -1 past the root, so the per-tree walk loads them without following p0
    pg->anc_depth = depth0 <= 4 ? 4 : depth0 <= 8 ? 8 : 0;
    pg->anc0.clear();
    if (pg->anc_depth > 0) {
        const int32_t D = pg->anc_depth;
        pg->anc0.assign((size_t)D * (size_t)n, -1);
        for (int64_t v = 0; v < n; ++v) {
            int32_t x = (int32_t)v;
            for (int32_t i = 0; i < D && x != root; ++i) {
                x = p0[(size_t)x];
                pg->anc0[(size_t)i * (size_t)n + (size_t)v] = x;
            }
        }
    }
    // per-vertex graph record for the sampler: offset, degree, first six neighbours
    std::vector<int32_t> &vrec = pg->vrec;
    vrec.assign((size_t)n * 8, -1);
    for (int64_t v = 0; v < n; ++v) {
        const int64_t a = off[(size_t)v], b = off[(size_t)v + 1];
        int32_t *r = &vrec[(size_t)v * 8];
        r[0] = (int32_t)a;
        r[1] = (int32_t)(b - a);
        for (int64_t k = 0; k < 6 && a + k < b; ++k) r[2 + k] = indices[a + k];
    }
    return KC_OK;
}

void free_graph_arrays(kc_graph *g) {
    dev_free(g->d_vrec);
    dev_free(g->d_anc0);
    g->d_anc0 = nullptr;
    g->anc_depth = 0;
    dev_free(g->d_off); dev_free(g->d_adj); dev_free(g->d_p0); dev_free(g->d_order);
    dev_free(g->d_pre0); dev_free(g->d_out0); dev_free(g->d_eoff); dev_free(g->d_elist);
    g->d_vrec = nullptr;
    g->d_off = nullptr; g->d_adj = g->d_p0 = g->d_order = g->d_pre0 = g->d_out0 = nullptr;
    g->d_eoff = g->d_elist = nullptr;
    g->graph_bytes = 0;
}

kc_status rebuild_graph(kc_graph *g, int32_t root, hipStream_t stream) {
    PreparedGraph pg;
    const kc_status st = prepare_graph(g->h_off, g->h_adj, root, g->tau0_kind, &g->h_tau0, &pg);
    if (st != KC_OK) return st;
    HIP_TRY(hipStreamSynchronize(stream));  // no running launch reads the old arrays
    free_graph_arrays(g);
    const int64_t n = (int64_t)g->h_off.size() - 1;
    g->n = n;
    g->two_m = g->h_off[(size_t)n];
    g->root = pg.root;
    g->depth0 = pg.depth0;
    g->nblk = pg.nblk;
    g->max_degree = 0;
    for (int64_t v = 0; v < n; ++v)
        g->max_degree = (int32_t)std::max<int64_t>(g->max_degree, g->h_off[(size_t)v + 1] - g->h_off[(size_t)v]);
    if (g->trav_opt == KC_TRAV_AUTO) g->traversal = pg.depth0 <= 12 ? KC_TRAV_WALK : KC_TRAV_SWEEP;
    g->bfs_order = pg.order;
    auto up = [&](auto **dst, const auto *src, size_t cnt) -> hipError_t {
        hipError_t e = dev_alloc(dst, cnt);
        if (e != hipSuccess) return e;
        g->graph_bytes += (int64_t)(cnt * sizeof(**dst));
        if (cnt == 0) return hipSuccess;
        return hipMemcpyAsync(*dst, src, cnt * sizeof(**dst), hipMemcpyHostToDevice, stream);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(&g->d_off, g->h_off.data(), g->h_off.size());
    if (e == hipSuccess) e = up(&g->d_adj, g->h_adj.data(), g->h_adj.size());
    if (e == hipSuccess) e = up(&g->d_p0, pg.p0.data(), pg.p0.size());
    const std::vector<int32_t> start_ord = start_order_of(pg.order, g->start_order);
    if (e == hipSuccess) e = up(&g->d_order, start_ord.data(), start_ord.size());
    if (e == hipSuccess) e = up(&g->d_pre0, pg.pre0.data(), pg.pre0.size());
    if (e == hipSuccess) e = up(&g->d_out0, pg.out0.data(), pg.out0.size());
    if (e == hipSuccess) e = up(&g->d_eoff, pg.eoff.data(), pg.eoff.size());
    if (e == hipSuccess) e = up(&g->d_elist, pg.elist.data(), pg.elist.size());
    if (e == hipSuccess) e = up(&g->d_vrec, reinterpret_cast<const int4 *>(pg.vrec.data()), (size_t)n * 2);
    if (e == hipSuccess && pg.anc_depth > 0) e = up(&g->d_anc0, pg.anc0.data(), pg.anc0.size());
    g->anc_depth = pg.anc_depth;
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? KC_ERR_NOMEM : KC_ERR_DEVICE, "upload failed: %s",
                    hipGetErrorString(e));
    return KC_OK;
}

kc_status refresh_resident_f(kc_graph *g, hipStream_t stream);

}  // namespace

extern "C" {

const char *kc_status_string(kc_status s) {
    switch (s) {
        case KC_OK: return "ok";
        case KC_ERR_INVALID: return "invalid argument or graph";
        case KC_ERR_DISCONNECTED: return "graph is not connected";
        case KC_ERR_NOMEM: return "out of memory";
        case KC_ERR_DEVICE: return "device error";
        case KC_ERR_OVERFLOW: return "graph too large for exact 64-bit tree values";
        case KC_ERR_LIMIT: return "step limit exceeded";
        case KC_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *kc_last_error(void) { return g_last_error.c_str(); }

kc_status kc_graph_create(int64_t n, const void *offsets, int offsets_are_i64, const int32_t *indices,
                          int32_t root, void *hip_stream, kc_graph **out) {
    g_last_error.clear();
    if (!out) return fail(KC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 2) return fail(KC_ERR_INVALID, "need at least 2 vertices (n=%lld)", (long long)n);
    if (n > (1ll << 31) - 1024) return fail(KC_ERR_UNSUPPORTED, "n=%lld exceeds 32-bit vertex ids", (long long)n);
    if (!offsets || !indices) return fail(KC_ERR_INVALID, "offsets/indices is NULL");
    hipStream_t stream = (hipStream_t)hip_stream;
    std::vector<int64_t> off((size_t)n + 1);
    if (offsets_are_i64) {
        std::memcpy(off.data(), offsets, sizeof(int64_t) * ((size_t)n + 1));
    } else {
        const int32_t *o32 = static_cast<const int32_t *>(offsets);
        for (int64_t i = 0; i <= n; ++i) off[(size_t)i] = o32[i];
    }
    if (off[0] != 0) return fail(KC_ERR_INVALID, "offsets[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (off[(size_t)i + 1] < off[(size_t)i]) return fail(KC_ERR_INVALID, "offsets decrease at row %lld", (long long)i);
    const int64_t nnz = off[(size_t)n];
    if (nnz >= (1ll << 31)) return fail(KC_ERR_OVERFLOW, "2m=%lld does not fit 31-bit volumes", (long long)nnz);
    int32_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) maxdeg = (int32_t)std::max<int64_t>(maxdeg, off[(size_t)v + 1] - off[(size_t)v]);
    // rows: neighbours in range, no self-loop, strictly ascending (the first bad row is reported)
    const int64_t bad_row = parallel_first(n, [&](int64_t lo, int64_t hi) -> int64_t {
        for (int64_t v = lo; v < hi; ++v) {
            const int64_t a = off[(size_t)v], b = off[(size_t)v + 1];
            for (int64_t e = a; e < b; ++e) {
                const int32_t u = indices[e];
                if (u < 0 || u >= n || u == v || (e > a && indices[e - 1] >= u)) return v;
            }
        }
        return -1;
    });
    if (bad_row >= 0) {
        const int64_t v = bad_row, a = off[(size_t)v], b = off[(size_t)v + 1];
        for (int64_t e = a; e < b; ++e) {
            const int32_t u = indices[e];
            if (u < 0 || u >= n) return fail(KC_ERR_INVALID, "neighbour %d of %lld out of range", u, (long long)v);
            if (u == v) return fail(KC_ERR_INVALID, "self-loop at %lld", (long long)v);
            if (e > a && indices[e - 1] >= u)
                return fail(KC_ERR_INVALID, "row %lld not strictly ascending (duplicate or unsorted)", (long long)v);
        }
    }
    if (maxdeg >= (1 << 20)) return fail(KC_ERR_UNSUPPORTED, "max degree %d >= 2^20", maxdeg);
    // every entry has its reverse entry (undirected); rows are valid at this point
    const int64_t no_rev = parallel_first(n, [&](int64_t lo, int64_t hi) -> int64_t {
        for (int64_t v = lo; v < hi; ++v)
            for (int64_t e = off[(size_t)v]; e < off[(size_t)v + 1]; ++e) {
                const int32_t u = indices[e];
                if (!std::binary_search(indices + off[(size_t)u], indices + off[(size_t)u + 1], (int32_t)v)) return v;
            }
        return -1;
    });
    if (no_rev >= 0) {
        for (int64_t e = off[(size_t)no_rev]; e < off[(size_t)no_rev + 1]; ++e) {
            const int32_t u = indices[e];
            if (!std::binary_search(indices + off[(size_t)u], indices + off[(size_t)u + 1], (int32_t)no_rev))
                return fail(KC_ERR_INVALID, "edge (%lld,%d) has no reverse entry", (long long)no_rev, u);
        }
    }
    kc_graph *g = new (std::nothrow) kc_graph();
    if (!g) return fail(KC_ERR_NOMEM, "host allocation failed");
    g->h_off = std::move(off);
    g->h_adj.assign(indices, indices + nnz);
    g->max_degree = maxdeg;
    // large sparse graphs (road-like: mean degree below 4) are bound by one
    // sample's rounds, and a chain table twice as large takes fewer of them; on
    // the 1M-point road-like graph 4,096 samples took 126 s with 2,048 chains
    // against 162 s with 1,024
    if (n >= 100000 && nnz < 4 * n) g->chains = 2048;
    const kc_status st = rebuild_graph(g, root, stream);
    if (st != KC_OK) {
        free_all(g);
        delete g;
        return st;
    }
    hipError_t e = dev_alloc(&g->d_ctl, 4);
    if (e == hipSuccess) e = dev_alloc(&g->d_red, 1);
    if (e != hipSuccess) {
        free_all(g);
        delete g;
        return fail(KC_ERR_NOMEM, "allocation failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return KC_OK;
}

kc_status kc_graph_destroy(kc_graph *g) {
    if (!g) return KC_OK;
    free_all(g);
    delete g;
    return KC_OK;
}

kc_status kc_graph_get_info(const kc_graph *g, kc_graph_info *info) {
    if (!g || !info) return fail(KC_ERR_INVALID, "NULL argument");
    info->n = g->n;
    info->two_m = g->two_m;
    info->root = g->root;
    info->depth0 = g->depth0;
    info->max_degree = g->max_degree;
    info->traversal = g->traversal;
    info->device_bytes = g->graph_bytes;
    info->tau0 = g->tau0_kind;
    info->sample_bytes = slot_bytes(g, true, g->traversal == KC_TRAV_SWEEP);
    info->chains = g->chains;
    return KC_OK;
}

kc_status kc_set_tau0(kc_graph *g, int kind, const int32_t *parent, void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (kind != KC_TAU0_BFS && kind != KC_TAU0_DFS && kind != KC_TAU0_GIVEN)
        return fail(KC_ERR_INVALID, "unknown tau0 rule %d", kind);
    if (kind == KC_TAU0_GIVEN && !parent) return fail(KC_ERR_INVALID, "tau0 parent array is NULL");
    hipStream_t stream = (hipStream_t)hip_stream;
    std::vector<int32_t> given;
    if (kind == KC_TAU0_GIVEN) given.assign(parent, parent + g->n);
    {
        PreparedGraph probe;  // validate before anything changes
        const kc_status st = prepare_graph(g->h_off, g->h_adj, g->root, kind, &given, &probe);
        if (st != KC_OK) return st;
    }
    const int32_t old_kind = g->tau0_kind;
    std::vector<int32_t> old_tau0 = g->h_tau0;
    g->tau0_kind = kind;
    g->h_tau0.swap(given);
    kc_status st = rebuild_graph(g, g->root, stream);
    // resident trees are unchanged; their f is taken over the new tau0 (Theorem 3.4)
    const bool was_stale = g->res_f_stale;
    if (st == KC_OK && g->res_count > 0) {
        g->res_f_stale = true;
        st = refresh_resident_f(g, stream);
    }
    if (st != KC_OK) {
        // put back the previous tau0; the f values taken over it are untouched
        const std::string err = g_last_error;
        g->tau0_kind = old_kind;
        g->h_tau0.swap(old_tau0);
        (void)rebuild_graph(g, g->root, stream);
        g->res_f_stale = was_stale;
        g_last_error = err;
        return st;
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return KC_OK;
}

kc_status kc_set_option(kc_graph *g, int option, int64_t value) {
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    switch (option) {
        case KC_OPT_WALKERS:
            if (value < 1 || value > 64) return fail(KC_ERR_INVALID, "walkers must be 1..64");
            g->walkers = (int32_t)value;
            return KC_OK;
        case KC_OPT_CHAINS:
            if (!kc::valid_chains((int)value)) return fail(KC_ERR_INVALID, "chains per sample must be 1024 or 2048");
            g->chains = (int32_t)value;
            return KC_OK;
        case KC_OPT_LEAN_LOOKS:
            if (value < 0 || value > 2) return fail(KC_ERR_INVALID, "lean looks must be 0, 1 or 2");
            g->lean_opt = (int32_t)value;
            return KC_OK;
        case KC_OPT_SLOTS:
            if (value < 0 || value > (1 << 20)) return fail(KC_ERR_INVALID, "slots must be 0..2^20");
            g->slots_opt = (int32_t)value;
            return KC_OK;
        case KC_OPT_TRAVERSAL:
            if (value == KC_TRAV_AUTO) g->traversal = g->depth0 <= 12 ? KC_TRAV_WALK : KC_TRAV_SWEEP;
            else if (value == KC_TRAV_WALK || value == KC_TRAV_SWEEP) g->traversal = (int32_t)value;
            else return fail(KC_ERR_INVALID, "unknown traversal %lld", (long long)value);
            g->trav_opt = (int32_t)value;
            return KC_OK;
        case KC_OPT_STEP_LIMIT:
            if (value < 0) return fail(KC_ERR_INVALID, "step limit must be >= 0");
            g->step_limit = value;
            return KC_OK;
        case KC_OPT_MEM_BUDGET:
            if (value < 0) return fail(KC_ERR_INVALID, "memory budget must be >= 0");
            g->mem_budget = value;
            g->ws_asked = std::min(g->ws_asked, g->ws_slots);  // the next launch re-fits to the new budget
            return KC_OK;
        case KC_OPT_MAINTENANCE:
            if (value != KC_MAINT_BASIC && value != KC_MAINT_IMPROVED)
                return fail(KC_ERR_INVALID, "maintenance must be KC_MAINT_BASIC or KC_MAINT_IMPROVED");
            if (g->res_count > 0 && value != g->maint)
                for (double w : g->res_w)
                    if (w != g->res_w[0])  // weighted trees are not a uniform set for basic maintenance
                        return fail(KC_ERR_INVALID, "the resident trees carry unequal weights; "
                                                    "re-initialise the set to change the maintenance");
            g->maint = (int32_t)value;
            return KC_OK;
        case KC_OPT_START_ORDER: {
            if (value < 0 || value > 2) return fail(KC_ERR_INVALID, "start order must be 0, 1 or 2");
            const std::vector<int32_t> ord = start_order_of(g->bfs_order, (int)value);
            HIP_TRY(hipMemcpy(g->d_order, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            g->start_order = (int32_t)value;
            return KC_OK;
        }
    }
    return fail(KC_ERR_INVALID, "unknown option %d", option);
}

kc_status kc_progress(const kc_graph *g, int64_t *samples_done) {
    if (!g || !samples_done) return KC_ERR_INVALID;
    int64_t sum = 0;
    for (int i = 0; i < g->progress_len; ++i) sum += __atomic_load_n(&g->h_progress[i], __ATOMIC_RELAXED);
    *samples_done = sum;
    return KC_OK;
}

kc_status kc_trim(kc_graph *g, void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));  // no launch still uses the workspace
    free_workspace(g);
    dev_free(g->d_f);
    dev_free(g->d_steps);
    dev_free(g->d_iters);
    g->d_f = g->d_steps = g->d_iters = nullptr;
    g->fbuf_len = 0;
    return KC_OK;
}

kc_status kc_reserve(kc_graph *g, int32_t count, void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (count < 1) return fail(KC_ERR_INVALID, "count must be >= 1");
    int want = g->slots_opt > 0 ? g->slots_opt : default_slots(g);
    want = std::min(want, count);
    int slots = 0;
    kc_status st = ensure_workspace(g, want, true, g->traversal == KC_TRAV_SWEEP, (hipStream_t)hip_stream, &slots);
    if (st != KC_OK) return st;
    st = ensure_fbuf(g, count);
    if (st != KC_OK) return st;
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    return KC_OK;
}

kc_status kc_sample_trees(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                          int32_t *parents_out, uint32_t *popcounts_out, int64_t *steps_out,
                          void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (count < 0 || first_sample < 0) return fail(KC_ERR_INVALID, "negative count or first sample");
    if (count == 0) return KC_OK;
    if (!parents_out) return fail(KC_ERR_INVALID, "parents_out is NULL");
    kc::RunParams rp{};
    rp.seed = seed;
    rp.first = first_sample;
    rp.count = count;
    rp.mode = kc::RUN_SAMPLE;
    rp.parents_out = parents_out;
    rp.cnt_out = popcounts_out;
    rp.steps_out = steps_out;
    return run_persistent(g, rp, (hipStream_t)hip_stream);
}

}  // extern "C"

// kappa and its standard error from the exact sums of a result (Theorem 3.3):
// kappa = sum f / (2 m count), one correctly rounded conversion and one
// division; std_error = the sample standard deviation of f / 2m over sqrt(count).
void kc_host::finish_result(int64_t two_m, kc_result *res) {
    const __int128 s1 = (__int128)(((unsigned __int128)(uint64_t)res->sum_f_hi << 64) | res->sum_f_lo);
    const unsigned __int128 s2 = ((unsigned __int128)res->sum_f2_hi << 64) | res->sum_f2_lo;
    const int64_t count = res->count;
    res->kappa = (double)s1 / (double)(two_m * count);
    if (count > 1) {
        const double mean = (double)s1 / (double)count;
        const double var = ((double)s2 - (double)count * mean * mean) / (double)(count - 1);
        res->std_error = std::sqrt(std::max(var, 0.0) / (double)count) / (double)two_m;
    } else {
        res->std_error = std::nan("");
    }
}

kc_status kc_host::finish_reduce(kc_graph *g, int32_t count, const int64_t *f, const int64_t *steps,
                               const int64_t *iters, kc_result *res, hipStream_t stream) {
    HIP_TRY(kc::launch_reduce(f, steps, iters, count, g->d_red, stream));
    kc::ReduceOut ro;
    HIP_TRY(hipMemcpyAsync(&ro, g->d_red, sizeof(ro), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    res->sum_f_lo = ro.sum_lo;
    res->sum_f_hi = ro.sum_hi;
    res->sum_f2_lo = ro.sq_lo;
    res->sum_f2_hi = ro.sq_hi;
    res->count = count;
    res->total_steps = ro.steps;
    res->sampler_iterations = ro.iters;
    finish_result(g->two_m, res);
    return KC_OK;
}

extern "C" {

kc_status kc_combine_results(const kc_graph *g, const kc_result *parts, int32_t k, kc_result *out) {
    g_last_error.clear();
    if (!g || !parts || !out) return fail(KC_ERR_INVALID, "NULL argument");
    if (k < 1) return fail(KC_ERR_INVALID, "need at least one result");
    unsigned __int128 s1 = 0, s2 = 0;
    kc_result r{};
    for (int32_t i = 0; i < k; ++i) {
        const kc_result &p = parts[i];
        if (p.count < 1) return fail(KC_ERR_INVALID, "result %d has no samples", i);
        s1 += ((unsigned __int128)(uint64_t)p.sum_f_hi << 64) | p.sum_f_lo;
        s2 += ((unsigned __int128)p.sum_f2_hi << 64) | p.sum_f2_lo;
        r.count += p.count;
        r.total_steps += p.total_steps;
        r.sampler_iterations += p.sampler_iterations;
    }
    r.sum_f_lo = (uint64_t)s1;
    r.sum_f_hi = (int64_t)(uint64_t)(s1 >> 64);
    r.sum_f2_lo = (uint64_t)s2;
    r.sum_f2_hi = (uint64_t)(s2 >> 64);
    finish_result(g->two_m, &r);
    *out = r;
    return KC_OK;
}

kc_status kc_estimate(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                      kc_result *result, int64_t *f_out, int64_t *steps_out, void *hip_stream) {
    g_last_error.clear();
    if (!g || !result) return fail(KC_ERR_INVALID, "NULL graph or result");
    if (count < 1 || first_sample < 0) return fail(KC_ERR_INVALID, "count must be >= 1");
    hipStream_t stream = (hipStream_t)hip_stream;
    int64_t *f = f_out, *steps = steps_out;
    kc_status st0 = ensure_fbuf(g, count);
    if (st0 != KC_OK) return st0;
    if (!f) f = g->d_f;
    if (!steps) steps = g->d_steps;
    kc::RunParams rp{};
    rp.seed = seed;
    rp.first = first_sample;
    rp.count = count;
    rp.mode = kc::RUN_ESTIMATE;
    rp.f_out = f;
    rp.steps_out = steps;
    rp.iters_out = g->d_iters;
    kc_status st = run_persistent(g, rp, stream);
    if (st != KC_OK) return st;
    return finish_reduce(g, count, f, steps, g->d_iters, result, stream);
}

kc_status kc_evaluate_trees(kc_graph *g, const int32_t *parents, int32_t count, int64_t *f_out,
                            void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (count < 0) return fail(KC_ERR_INVALID, "negative count");
    if (count == 0) return KC_OK;
    if (!parents || !f_out) return fail(KC_ERR_INVALID, "parents/f_out is NULL");
    kc::RunParams rp{};
    rp.count = count;
    rp.mode = kc::RUN_EVALUATE;
    rp.parents_in = parents;
    rp.f_out = f_out;
    return run_persistent(g, rp, (hipStream_t)hip_stream);
}


kc_status kc_samples_init(kc_graph *g, uint64_t seed, int32_t count, void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (count < 1) return fail(KC_ERR_INVALID, "count must be >= 1");
    hipStream_t stream = (hipStream_t)hip_stream;
    dev_free(g->d_res_par);
    dev_free(g->d_res_f);
    g->d_res_par = nullptr;
    g->d_res_f = nullptr;
    g->res_count = 0;
    g->res_ids.clear();
    dev_free(g->d_res_f_alt);
    g->d_res_f_alt = nullptr;
    g->res_f_stale = false;
    HIP_TRY(dev_alloc(&g->d_res_par, (size_t)count * (size_t)g->n));
    HIP_TRY(dev_alloc(&g->d_res_f, (size_t)count));
    HIP_TRY(dev_alloc(&g->d_res_f_alt, (size_t)count));
    kc_status st = kc_sample_trees(g, seed, 0, count, g->d_res_par, nullptr, nullptr, hip_stream);
    if (st != KC_OK) return st;
    st = kc_evaluate_trees(g, g->d_res_par, count, g->d_res_f, hip_stream);
    if (st != KC_OK) return st;
    HIP_TRY(hipStreamSynchronize(stream));
    g->res_count = count;
    g->res_seed = seed;
    g->res_next = count;
    g->res_ids.resize((size_t)count);
    for (int32_t i = 0; i < count; ++i) g->res_ids[(size_t)i] = i;
    g->res_serial = 0;
    g->res_w.assign((size_t)count, 1.0 / (double)count);
    return KC_OK;
}

kc_status kc_samples_query(kc_graph *g, kc_result *result, void *hip_stream) {
    g_last_error.clear();
    if (!g || !result) return fail(KC_ERR_INVALID, "NULL graph or result");
    if (g->res_count < 1) return fail(KC_ERR_INVALID, "no resident samples (call kc_samples_init)");
    hipStream_t stream = (hipStream_t)hip_stream;
    // f from before the last update is never reduced: a failed recomputation is retried here
    kc_status st = refresh_resident_f(g, stream);
    if (st != KC_OK) return st;
    st = finish_reduce(g, g->res_count, g->d_res_f, nullptr, nullptr, result, stream);
    if (st != KC_OK || g->maint != KC_MAINT_IMPROVED) return st;
    // Algorithm 3: kappa = sum_t w_t f_t / 2m, weights summing to one, in slot order
    std::vector<int64_t> f((size_t)g->res_count);
    HIP_TRY(hipMemcpyAsync(f.data(), g->d_res_f, f.size() * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const double two_m = (double)g->two_m;
    double k = 0.0;
    for (size_t t = 0; t < f.size(); ++t) k += g->res_w[t] * (double)f[t];
    k /= two_m;
    double v = 0.0;
    for (size_t t = 0; t < f.size(); ++t) {
        const double d = (double)f[t] / two_m - k;
        v += g->res_w[t] * g->res_w[t] * d * d;
    }
    result->kappa = k;
    result->std_error = std::sqrt(v);
    return KC_OK;
}

kc_status kc_samples_weights(const kc_graph *g, double *w_out) {
    g_last_error.clear();
    if (!g || !w_out) return fail(KC_ERR_INVALID, "NULL argument");
    if (g->res_count < 1) return fail(KC_ERR_INVALID, "no resident samples (call kc_samples_init)");
    std::memcpy(w_out, g->res_w.data(), g->res_w.size() * sizeof(double));
    return KC_OK;
}

kc_status kc_samples_get(kc_graph *g, int32_t *parents_out, int64_t *f_out, int64_t *ids_out,
                         void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    hipStream_t stream = (hipStream_t)hip_stream;
    if (f_out) {
        const kc_status st = refresh_resident_f(g, stream);
        if (st != KC_OK) return st;
    }
    const size_t c = (size_t)g->res_count;
    if (parents_out && c)
        HIP_TRY(hipMemcpyAsync(parents_out, g->d_res_par, c * (size_t)g->n * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, stream));
    if (f_out && c) HIP_TRY(hipMemcpyAsync(f_out, g->d_res_f, c * sizeof(int64_t), hipMemcpyDeviceToDevice, stream));
    if (ids_out && c) std::memcpy(ids_out, g->res_ids.data(), c * sizeof(int64_t));
    HIP_TRY(hipStreamSynchronize(stream));
    return KC_OK;
}

static kc_status ism_deletion(kc_graph *g, int32_t a, int32_t b, int32_t *changed, hipStream_t stream, bool last);

// Moves g to a new CSR and keeps the old one; undo() puts back the old CSR
// and tau0 rule and rebuilds every per-graph array, so that an update that
// fails after the switch leaves the graph as it was.  It returns the status
// of the failure and keeps its message.
struct GraphSwitch {
    kc_graph *g;
    std::vector<int64_t> old_off;
    std::vector<int32_t> old_adj;
    int32_t old_kind;
    std::vector<int32_t> old_tau0;
    GraphSwitch(kc_graph *g_, std::vector<int64_t> &&noff, std::vector<int32_t> &&nadj)
        : g(g_), old_kind(g_->tau0_kind), old_tau0(g_->h_tau0) {
        old_off.swap(g->h_off);
        old_adj.swap(g->h_adj);
        g->h_off = std::move(noff);
        g->h_adj = std::move(nadj);
    }
    kc_status undo(kc_status st, hipStream_t stream) {
        const std::string err = g_last_error;
        g->h_off.swap(old_off);
        g->h_adj.swap(old_adj);
        g->tau0_kind = old_kind;
        g->h_tau0 = old_tau0;
        if (rebuild_graph(g, g->root, stream) != KC_OK) {
            g_last_error = err + "; restoring the previous graph failed too: " + g_last_error;
            return st;
        }
        g_last_error = err;
        return st;
    }
};

// flags[t] = 1 for the resident trees that contain one of the edges {eu[k], ev[k]}.
static std::vector<uint8_t> trees_with_edges(kc_graph *g, const std::vector<int32_t> &eu,
                                             const std::vector<int32_t> &ev, hipStream_t stream, kc_status *st) {
    std::vector<uint8_t> flags((size_t)g->res_count, 0);
    *st = KC_OK;
    DevTmp<int32_t> d_eu, d_ev;
    DevTmp<uint8_t> d_flags;
    hipError_t e = d_eu.alloc(eu.size(), stream);
    if (e == hipSuccess) e = d_ev.alloc(ev.size(), stream);
    if (e == hipSuccess) e = d_flags.alloc((size_t)g->res_count, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_eu.p, eu.data(), eu.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ev.p, ev.data(), ev.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_flags.p, 0, (size_t)g->res_count, stream);
    if (e == hipSuccess)
        e = kc::launch_flag_trees(g->d_res_par, g->res_count, g->n, d_eu.p, d_ev.p, (int32_t)eu.size(), d_flags.p,
                                  stream);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), d_flags.p, flags.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        *st = fail(e == hipErrorOutOfMemory ? KC_ERR_NOMEM : KC_ERR_DEVICE, "flagging trees failed: %s",
                   hipGetErrorString(e));
    return flags;
}

// A device copy of resident rows, to put them back if an update fails after
// changing them in place.
struct RowBackup {
    DevTmp<int32_t> buf;
    std::vector<int32_t> rows;
    kc_status save(kc_graph *g, const std::vector<int32_t> &r, hipStream_t stream) {
        rows = r;
        if (rows.empty()) return KC_OK;
        HIP_TRY(buf.alloc(rows.size() * (size_t)g->n, stream));
        for (size_t i = 0; i < rows.size(); ++i)
            HIP_TRY(hipMemcpyAsync(buf.p + i * (size_t)g->n, g->d_res_par + (size_t)rows[i] * (size_t)g->n,
                                   (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
        return KC_OK;
    }
    void restore(kc_graph *g, hipStream_t stream) {
        for (size_t i = 0; i < rows.size(); ++i)
            (void)hipMemcpyAsync(g->d_res_par + (size_t)rows[i] * (size_t)g->n, buf.p + i * (size_t)g->n,
                                 (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream);
        (void)hipStreamSynchronize(stream);
    }
};

// A run of deletions, applied at once (Algorithm 2, deletion case).
static kc_status apply_deletions(kc_graph *g, const int32_t *u, const int32_t *v, int32_t count,
                                 int32_t *resampled, hipStream_t stream) {
    const int64_t n = g->n;
    // validate: deletions of distinct existing edges
    std::vector<std::pair<int32_t, int32_t>> del;
    del.reserve((size_t)count);
    for (int32_t k = 0; k < count; ++k) {
        int32_t a = u[k], b = v[k];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(KC_ERR_INVALID, "bad edge (%d,%d)", a, b);
        if (a > b) std::swap(a, b);
        if (!std::binary_search(g->h_adj.begin() + g->h_off[(size_t)a], g->h_adj.begin() + g->h_off[(size_t)a + 1], b))
            return fail(KC_ERR_INVALID, "edge (%d,%d) is not in the graph", a, b);
        del.emplace_back(a, b);
    }
    std::sort(del.begin(), del.end());
    if (std::adjacent_find(del.begin(), del.end()) != del.end()) return fail(KC_ERR_INVALID, "duplicate edge in batch");
    auto deleted = [&](int32_t a, int32_t b) {
        if (a > b) std::swap(a, b);
        return std::binary_search(del.begin(), del.end(), std::make_pair(a, b));
    };
    // the graph after the batch (G')
    std::vector<int64_t> noff((size_t)n + 1, 0);
    std::vector<int32_t> nadj;
    nadj.reserve(g->h_adj.size() - 2 * del.size());
    for (int64_t x = 0; x < n; ++x) {
        for (int64_t e = g->h_off[(size_t)x]; e < g->h_off[(size_t)x + 1]; ++e) {
            const int32_t y = g->h_adj[(size_t)e];
            if (!deleted((int32_t)x, y)) nadj.push_back(y);
        }
        noff[(size_t)x + 1] = (int64_t)nadj.size();
    }
    // a caller's tau0 that loses an edge gives way to the BFS rule
    int kind = g->tau0_kind;
    if (kind == KC_TAU0_GIVEN)
        for (const auto &e : del)
            if (g->h_tau0[(size_t)e.first] == e.second || g->h_tau0[(size_t)e.second] == e.first) kind = KC_TAU0_BFS;
    {
        PreparedGraph probe;  // G' must stay connected (section 2.1); nothing changes if not
        const kc_status st = prepare_graph(noff, nadj, g->root, kind, &g->h_tau0, &probe);
        if (st != KC_OK) return st;
    }
    if (g->maint == KC_MAINT_IMPROVED && g->res_count > 0) {
        // Algorithm 3 takes one edge at a time; every intermediate graph contains
        // the final one, so it is connected too
        for (int32_t k = 0; k < count; ++k) {
            const kc_status st = ism_deletion(g, u[k], v[k], resampled, stream, k == count - 1);
            if (st != KC_OK) return st;
        }
        return KC_OK;
    }
    // resident trees that use a deleted edge (Algorithm 2, deletion: they are
    // replaced; the others are uniform spanning trees of G' already, Theorem 4.2)
    std::vector<int32_t> redo;
    kc_status st0 = KC_OK;
    if (g->res_count > 0) {
        std::vector<int32_t> eu(del.size()), ev(del.size());
        for (size_t k = 0; k < del.size(); ++k) { eu[k] = del[k].first; ev[k] = del[k].second; }
        const std::vector<uint8_t> flags = trees_with_edges(g, eu, ev, stream, &st0);
        if (st0 != KC_OK) return st0;
        for (int32_t t = 0; t < g->res_count; ++t)
            if (flags[(size_t)t]) redo.push_back(t);
    }
    // switch to G'
    GraphSwitch sw(g, std::move(noff), std::move(nadj));
    if (kind != g->tau0_kind) {
        g->tau0_kind = kind;
        g->h_tau0.clear();
    }
    kc_status st = rebuild_graph(g, g->root, stream);
    if (st != KC_OK) return sw.undo(st, stream);
    if (g->res_count > 0) {
        // fresh trees of G' for the replaced ones: the next unused sample indices, in slot order
        const int32_t k = (int32_t)redo.size();
        if (k > 0) {
            DevTmp<int32_t> tmp;
            hipError_t e = tmp.alloc((size_t)k * (size_t)n, stream);
            if (e != hipSuccess) return sw.undo(fail(KC_ERR_NOMEM, "allocation failed: %s", hipGetErrorString(e)), stream);
            st = kc_sample_trees(g, g->res_seed, g->res_next, k, tmp.p, nullptr, nullptr, (void *)stream);
            if (st != KC_OK) return sw.undo(st, stream);
            // from here on nothing can fail before the set is consistent with G'
            for (int32_t i = 0; i < k; ++i) {
                HIP_TRY(hipMemcpyAsync(g->d_res_par + (size_t)redo[(size_t)i] * (size_t)n, tmp.p + (size_t)i * (size_t)n,
                                       (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
                g->res_ids[(size_t)redo[(size_t)i]] = g->res_next + i;
            }
            HIP_TRY(hipStreamSynchronize(stream));
            g->res_next += k;
        }
        // every tree's f on G' (degrees, 2m and tau0 changed), at the end of the call
        g->res_f_stale = true;
        if (resampled) *resampled += k;
    }
    return KC_OK;
}

// The CSR with the undirected edge {a, b} added (rows stay ascending).
static void csr_with_edge(const std::vector<int64_t> &off, const std::vector<int32_t> &adj, int32_t a, int32_t b,
                          std::vector<int64_t> *noff, std::vector<int32_t> *nadj) {
    const int64_t n = (int64_t)off.size() - 1;
    noff->assign((size_t)n + 1, 0);
    nadj->clear();
    nadj->reserve(adj.size() + 2);
    for (int64_t x = 0; x < n; ++x) {
        const int32_t add = x == a ? b : x == b ? a : -1;
        bool done = add < 0;
        for (int64_t e = off[(size_t)x]; e < off[(size_t)x + 1]; ++e) {
            const int32_t y = adj[(size_t)e];
            if (!done && add < y) { nadj->push_back(add); done = true; }
            nadj->push_back(y);
        }
        if (!done) nadj->push_back(add);
        (*noff)[(size_t)x + 1] = (int64_t)nadj->size();
    }
}

// The CSR with the undirected edge {a, b} removed.
static void csr_without_edge(const std::vector<int64_t> &off, const std::vector<int32_t> &adj, int32_t a,
                             int32_t b, std::vector<int64_t> *noff, std::vector<int32_t> *nadj) {
    const int64_t n = (int64_t)off.size() - 1;
    noff->assign((size_t)n + 1, 0);
    nadj->clear();
    nadj->reserve(adj.size());
    for (int64_t x = 0; x < n; ++x) {
        for (int64_t e = off[(size_t)x]; e < off[(size_t)x + 1]; ++e) {
            const int32_t y = adj[(size_t)e];
            if (!((x == a && y == b) || (x == b && y == a))) nadj->push_back(y);
        }
        (*noff)[(size_t)x + 1] = (int64_t)nadj->size();
    }
}

// R(a, b) on the current graph from the resident trees: per tree, the
// signed count of the edges of a fixed breadth-first a -> b path that the
// tree's own a -> b path uses (its mean over uniform trees is R(a, b)).
static kc_status path_currents(kc_graph *g, int32_t a, int32_t b, std::vector<int64_t> *c, hipStream_t stream) {
    const std::vector<int32_t> path = reference_path(g->h_off, g->h_adj, a, b);
    if (path.size() < 2) return fail(KC_ERR_DEVICE, "no path between %d and %d", a, b);
    DevTmp<int32_t> d_path;
    DevTmp<int64_t> d_c;
    HIP_TRY(d_path.alloc(path.size(), stream));
    HIP_TRY(d_c.alloc((size_t)g->res_count, stream));
    HIP_TRY(hipMemcpyAsync(d_path.p, path.data(), path.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    kc::RunParams rp{};
    rp.count = g->res_count;
    rp.mode = kc::RUN_CURRENT;
    rp.parents_in = g->d_res_par;
    rp.f_out = d_c.p;
    rp.path = d_path.p;
    rp.path_len = (int32_t)path.size();
    kc_status st = run_persistent(g, rp, stream);
    c->assign((size_t)g->res_count, 0);
    if (st == KC_OK) {
        const hipError_t e = hipMemcpy(c->data(), d_c.p, c->size() * sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = fail(KC_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
    }
    return st;
}

// One insertion (Algorithm 2, insertion case; Theorem 4.1).
static kc_status apply_insertion(kc_graph *g, int32_t a, int32_t b, int32_t *resampled, hipStream_t stream) {
    const int64_t n = g->n;
    if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(KC_ERR_INVALID, "bad edge (%d,%d)", a, b);
    if (std::binary_search(g->h_adj.begin() + g->h_off[(size_t)a], g->h_adj.begin() + g->h_off[(size_t)a + 1], b))
        return fail(KC_ERR_INVALID, "edge (%d,%d) is already in the graph", a, b);
    if (g->two_m + 2 >= (1ll << 31)) return fail(KC_ERR_OVERFLOW, "2m would reach 2^31");
    // G' = G + (a, b)
    std::vector<int64_t> noff;
    std::vector<int32_t> nadj;
    csr_with_edge(g->h_off, g->h_adj, a, b, &noff, &nadj);
    {
        PreparedGraph probe;  // tau0 of G' must pass the overflow bound; nothing changes if not
        const kc_status st = prepare_graph(noff, nadj, g->root, g->tau0_kind, &g->h_tau0, &probe);
        if (st != KC_OK) return st;
    }
    std::vector<int32_t> redo;
    if (g->res_count > 0) {
        std::vector<int64_t> c;
        kc_status st = path_currents(g, a, b, &c, stream);
        if (st != KC_OK) return st;
        int64_t csum = 0;
        for (int64_t x : c) csum += x;
        const double rhat = (double)csum / (double)g->res_count;
        // R_G'(e) = R / (1 + R), Theorem 4.1; an estimate R <= 0 (possible for a
        // small set) means no tree is replaced
        const double p = rhat > 0.0 ? rhat / (1.0 + rhat) : 0.0;
        for (int32_t t = 0; t < g->res_count; ++t)
            if (update_uniform(g->res_seed, (uint32_t)t, (uint32_t)g->res_serial) < p) redo.push_back(t);
    }
    GraphSwitch sw(g, std::move(noff), std::move(nadj));
    kc_status st = rebuild_graph(g, g->root, stream);
    if (st != KC_OK) return sw.undo(st, stream);
    if (g->res_count > 0) {
        const int32_t k = (int32_t)redo.size();
        if (k > 0) {
            // uniform spanning trees of G' through (a, b): a and b start in the tree
            DevTmp<int32_t> tmp;
            hipError_t e = tmp.alloc((size_t)k * (size_t)n, stream);
            if (e != hipSuccess) return sw.undo(fail(KC_ERR_NOMEM, "allocation failed: %s", hipGetErrorString(e)), stream);
            kc::RunParams rp{};
            rp.seed = g->res_seed;
            rp.first = g->res_next;
            rp.count = k;
            rp.mode = kc::RUN_SAMPLE;
            rp.parents_out = tmp.p;
            rp.root_u = a;
            rp.root_v = b;
            st = run_persistent(g, rp, stream);
            if (st == KC_OK) {
                e = kc::launch_reroot(tmp.p, k, n, a, b, g->root, stream);
                if (e != hipSuccess) st = fail(KC_ERR_DEVICE, "reroot failed: %s", hipGetErrorString(e));
            }
            if (st != KC_OK) return sw.undo(st, stream);
            for (int32_t i = 0; i < k; ++i) {
                HIP_TRY(hipMemcpyAsync(g->d_res_par + (size_t)redo[(size_t)i] * (size_t)n, tmp.p + (size_t)i * (size_t)n,
                                       (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
                g->res_ids[(size_t)redo[(size_t)i]] = g->res_next + i;
            }
            HIP_TRY(hipStreamSynchronize(stream));
            g->res_next += k;
        }
        g->res_f_stale = true;
        g->res_serial += 1;
        if (resampled) *resampled += k;
    }
    return KC_OK;
}

// Per-tree integers of an improved-maintenance step, computed on the device for
// the resident trees `rows` (DEVICE copies made here).
static kc_status ism_link_cut(kc_graph *g, const std::vector<int32_t> &rows, int32_t a, int32_t b, int relink,
                              std::vector<int64_t> *d, hipStream_t stream) {
    const int32_t k = (int32_t)rows.size();
    d->assign((size_t)k, 0);
    if (k == 0) return KC_OK;
    DevTmp<int32_t> d_rows;
    DevTmp<int64_t> d_d;
    HIP_TRY(d_rows.alloc((size_t)k, stream));
    HIP_TRY(d_d.alloc((size_t)k, stream));
    HIP_TRY(hipMemcpyAsync(d_rows.p, rows.data(), (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(kc::launch_reset_ctl(g->d_ctl, stream));
    HIP_TRY(kc::launch_link_cut(g->d_res_par, d_rows.p, k, g->n, a, b, g->res_seed, (uint32_t)g->res_serial, relink,
                                d_d.p, g->d_ctl, stream));
    int32_t ctl[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(ctl, g->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(d->data(), d_d.p, (size_t)k * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (ctl[1] != 0) return fail(KC_ERR_INVALID, "resident tree %d is not a tree rooted at %d", rows[(size_t)ctl[2]], g->root);
    return KC_OK;
}

static kc_status ism_cross(kc_graph *g, const std::vector<int32_t> &rows, int32_t a, int32_t b, int relink,
                           std::vector<int64_t> *d, hipStream_t stream) {
    const int32_t k = (int32_t)rows.size();
    d->assign((size_t)k, 0);
    if (k == 0) return KC_OK;
    DevTmp<int32_t> d_rows;
    DevTmp<int64_t> d_d;
    HIP_TRY(d_rows.alloc((size_t)k, stream));
    HIP_TRY(d_d.alloc((size_t)k, stream));
    HIP_TRY(hipMemcpyAsync(d_rows.p, rows.data(), (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    kc::RunParams rp{};
    rp.count = k;
    rp.mode = kc::RUN_CROSS;
    rp.seed = g->res_seed;
    rp.parents_in = g->d_res_par;
    rp.parents_mut = g->d_res_par;
    rp.rows = d_rows.p;
    rp.f_out = d_d.p;
    rp.cut_u = a;
    rp.cut_v = b;
    rp.relink = relink;
    rp.serial = (uint32_t)g->res_serial;
    kc_status st = run_persistent(g, rp, stream);
    if (st == KC_OK) {
        const hipError_t e = hipMemcpy(d->data(), d_d.p, (size_t)k * sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = fail(KC_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
    }
    return st;
}

static void normalise(std::vector<double> &w, const std::vector<int32_t> &group, double target) {
    double s = 0.0;
    for (int32_t t : group) s += w[(size_t)t];
    for (int32_t t : group) w[(size_t)t] *= target / s;
}

// One insertion by improved sample maintenance (Algorithm 3; Theorem 4.4).
static kc_status ism_insertion(kc_graph *g, int32_t a, int32_t b, int32_t *changed, hipStream_t stream) {
    const int64_t n = g->n;
    if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(KC_ERR_INVALID, "bad edge (%d,%d)", a, b);
    if (std::binary_search(g->h_adj.begin() + g->h_off[(size_t)a], g->h_adj.begin() + g->h_off[(size_t)a + 1], b))
        return fail(KC_ERR_INVALID, "edge (%d,%d) is already in the graph", a, b);
    if (g->two_m + 2 >= (1ll << 31)) return fail(KC_ERR_OVERFLOW, "2m would reach 2^31");
    std::vector<int64_t> noff;
    std::vector<int32_t> nadj;
    csr_with_edge(g->h_off, g->h_adj, a, b, &noff, &nadj);
    {
        PreparedGraph probe;
        const kc_status st = prepare_graph(noff, nadj, g->root, g->tau0_kind, &g->h_tau0, &probe);
        if (st != KC_OK) return st;
    }
    const int32_t count = g->res_count;
    // R(a, b) from the weighted set; R' = R / (1 + R) is the share of G''s trees through e
    std::vector<int64_t> c;
    kc_status st = path_currents(g, a, b, &c, stream);
    if (st != KC_OK) return st;
    double rhat = 0.0;
    for (int32_t t = 0; t < count; ++t) rhat += g->res_w[(size_t)t] * (double)c[(size_t)t];
    const double rp = rhat > 0.0 ? rhat / (1.0 + rhat) : 0.0;  // as in the basic case
    const int32_t k = (int32_t)std::min<double>((double)count, std::ceil(rp * (double)count));
    // ceil(R' |S|) trees chosen uniformly: the smallest replacement draws
    std::vector<std::pair<double, int32_t>> key((size_t)count);
    for (int32_t t = 0; t < count; ++t)
        key[(size_t)t] = {update_uniform(g->res_seed, (uint32_t)t, (uint32_t)g->res_serial), t};
    std::sort(key.begin(), key.end());
    std::vector<int32_t> chosen, rest;
    for (int32_t i = 0; i < count; ++i) (i < k ? chosen : rest).push_back(key[(size_t)i].second);
    std::sort(chosen.begin(), chosen.end());
    std::sort(rest.begin(), rest.end());
    // link-cut in place (graph-independent); d(tau) = tree path length between a and b.
    // The chosen rows are saved first, so that a failure changes nothing.
    RowBackup saved;
    st = saved.save(g, chosen, stream);
    if (st != KC_OK) return st;
    std::vector<int64_t> d_old, d_new;
    st = ism_link_cut(g, chosen, a, b, 1, &d_old, stream);
    if (st != KC_OK) {
        saved.restore(g, stream);
        return st;
    }
    GraphSwitch sw(g, std::move(noff), std::move(nadj));
    st = rebuild_graph(g, g->root, stream);
    // d(tau_e): edges of G that join the two parts of tau_e - e (those of G' minus e itself)
    if (st == KC_OK) st = ism_cross(g, chosen, a, b, 0, &d_new, stream);
    if (st != KC_OK) {
        saved.restore(g, stream);
        return sw.undo(st, stream);
    }
    for (size_t i = 0; i < chosen.size(); ++i)
        g->res_w[(size_t)chosen[i]] *= (double)d_old[i] / (double)(d_new[i] - 1);
    if (!chosen.empty() && !rest.empty()) {
        normalise(g->res_w, chosen, rp);
        normalise(g->res_w, rest, 1.0 - rp);
    } else {
        normalise(g->res_w, chosen.empty() ? rest : chosen, 1.0);
    }
    g->res_f_stale = true;
    g->res_serial += 1;
    if (changed) *changed += k;
    return KC_OK;
}

// The device CSR of an intermediate graph of a deletion run: cut-link and the
// tree numbering read only the row offsets and neighbours, and the rows only
// shrink, so they are copied into the arrays of the last full rebuild.
static kc_status upload_csr_only(kc_graph *g, hipStream_t stream) {
    HIP_TRY(hipStreamSynchronize(stream));  // no running launch reads the old rows
    HIP_TRY(hipMemcpyAsync(g->d_off, g->h_off.data(), g->h_off.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipMemcpyAsync(g->d_adj, g->h_adj.data(), g->h_adj.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    g->two_m = g->h_off[(size_t)g->n];
    return KC_OK;
}

// One deletion by improved sample maintenance (Algorithm 3; Theorem 4.5); the
// graph stays connected (checked by the caller for the whole run).  Only the
// run's last edge rebuilds tau0 and the other per-graph arrays.
static kc_status ism_deletion(kc_graph *g, int32_t a, int32_t b, int32_t *changed, hipStream_t stream, bool last) {
    const int32_t count = g->res_count;
    std::vector<int32_t> hit;
    {
        kc_status st0 = KC_OK;
        const std::vector<uint8_t> flags = trees_with_edges(g, {a}, {b}, stream, &st0);
        if (st0 != KC_OK) return st0;
        for (int32_t t = 0; t < count; ++t)
            if (flags[(size_t)t]) hit.push_back(t);
    }
    RowBackup saved;  // cut-link rewrites these rows in place; a failure puts them back
    {
        const kc_status st0 = saved.save(g, hit, stream);
        if (st0 != KC_OK) return st0;
    }
    double w_org = 0.0;
    for (int32_t t : hit) w_org += g->res_w[(size_t)t];
    std::vector<int64_t> noff;
    std::vector<int32_t> nadj;
    csr_without_edge(g->h_off, g->h_adj, a, b, &noff, &nadj);
    GraphSwitch sw(g, std::move(noff), std::move(nadj));
    if (g->tau0_kind == KC_TAU0_GIVEN && (g->h_tau0[(size_t)a] == b || g->h_tau0[(size_t)b] == a)) {
        g->tau0_kind = KC_TAU0_BFS;
        g->h_tau0.clear();
    }
    kc_status st = last ? rebuild_graph(g, g->root, stream) : upload_csr_only(g, stream);
    // cut-link in place; d(tau) = edges of G' that join the two parts of tau - e
    std::vector<int64_t> d_old, d_new;
    if (st == KC_OK) st = ism_cross(g, hit, a, b, 1, &d_old, stream);
    // d(tau') = tree path length between a and b in the new tree
    if (st == KC_OK) st = ism_link_cut(g, hit, a, b, 0, &d_new, stream);
    if (st != KC_OK) {
        saved.restore(g, stream);
        return sw.undo(st, stream);
    }
    for (size_t i = 0; i < hit.size(); ++i) g->res_w[(size_t)hit[i]] *= (double)d_old[i] / (double)d_new[i];
    if (!hit.empty()) normalise(g->res_w, hit, w_org);
    g->res_f_stale = true;
    g->res_serial += 1;
    if (changed) *changed += (int32_t)hit.size();
    return KC_OK;
}

kc_status kc_apply_updates(kc_graph *g, const int32_t *u, const int32_t *v, const uint8_t *is_insert,
                           int32_t count, int32_t *resampled, void *hip_stream) {
    g_last_error.clear();
    if (!g) return fail(KC_ERR_INVALID, "NULL graph");
    if (count < 0 || (count > 0 && (!u || !v))) return fail(KC_ERR_INVALID, "bad update arrays");
    if (resampled) *resampled = 0;
    hipStream_t stream = (hipStream_t)hip_stream;
    int32_t k = 0;
    kc_status st = KC_OK;
    while (k < count && st == KC_OK) {
        if (is_insert && is_insert[k]) {
            st = g->maint == KC_MAINT_IMPROVED && g->res_count > 0 ? ism_insertion(g, u[k], v[k], resampled, stream)
                                                                   : apply_insertion(g, u[k], v[k], resampled, stream);
            ++k;
        } else {
            int32_t e = k;
            while (e < count && !(is_insert && is_insert[e])) ++e;
            st = apply_deletions(g, u + k, v + k, e - k, resampled, stream);
            k = e;
        }
    }
    // f of every resident tree on the graph as it now stands (no update reads f,
    // so it is computed once per call), also when a later update failed
    if (g->res_f_stale && g->res_count > 0) {
        const std::string err = g_last_error;
        const kc_status st2 = refresh_resident_f(g, stream);
        if (st2 == KC_OK) {
            if (st != KC_OK) g_last_error = err;
        } else if (st == KC_OK) {
            st = st2;  // f stays marked stale: a query recomputes it or reports the failure
        }
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return st;
}

}  // extern "C"

namespace {

// f of every resident tree on the current graph, evaluated into the spare
// buffer and swapped in only when the whole evaluation succeeded, so that a
// failure leaves the previous values and the stale mark in place.
kc_status refresh_resident_f(kc_graph *g, hipStream_t stream) {
    if (!g->res_f_stale || g->res_count < 1) return KC_OK;
    const kc_status st = kc_evaluate_trees(g, g->d_res_par, g->res_count, g->d_res_f_alt, (void *)stream);
    if (st != KC_OK) return st;
    std::swap(g->d_res_f, g->d_res_f_alt);
    g->res_f_stale = false;
    return KC_OK;
}

}  // namespace
