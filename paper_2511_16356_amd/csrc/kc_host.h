// kc_host.h -- the library's host-side graph object and the launch helpers
// shared by the host source files (kc_host.cpp and the entry points kept in
// their own files).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/kc.h"
#include "kc_internal.h"

struct PreparedGraph {
    int32_t root = -1, depth0 = 0, nblk = 0, anc_depth = 0;
    std::vector<int32_t> order, p0, pre0, out0, eoff, elist, vrec, anc0;
};

struct kc_graph {
    int64_t n = 0, two_m = 0;
    int32_t root = -1, depth0 = 0, max_degree = 0;
    int32_t traversal = KC_TRAV_WALK;
    int32_t walkers = 64;
    int32_t chains = 1024;
    int32_t lean_opt = 0;  // KC_OPT_LEAN_LOOKS: 0 by mean degree, 1 off, 2 on
    int32_t slots_opt = 0;
    int32_t trav_opt = KC_TRAV_AUTO;
    int64_t step_limit = 0;
    int64_t mem_budget = 0;
    int64_t graph_bytes = 0;
    int32_t nblk = 0;
    int32_t start_order = 2;
    int32_t tau0_kind = KC_TAU0_BFS;  // rule that builds tau0 on every (re)build
    std::vector<int32_t> h_tau0;     // the caller's tau0 when tau0_kind == KC_TAU0_GIVEN
    std::vector<int32_t> bfs_order;  // host copy of the BFS order from the root
    std::vector<int64_t> h_off;      // host copy of the current CSR
    std::vector<int32_t> h_adj;
    // resident sample set (kc_samples_init / kc_apply_updates)
    int32_t res_count = 0;
    uint64_t res_seed = 0;
    int64_t res_next = 0;             // next unused sample index
    int64_t res_serial = 0;           // basic: insertions applied so far; improved: single-edge
                                      // updates applied so far (the counter of their draws)
    int32_t maint = KC_MAINT_BASIC;   // sample maintenance of the resident set
    std::vector<double> res_w;        // improved maintenance: weight of each tree (sum 1)
    bool res_f_stale = false;         // the graph changed since d_res_f was computed
    std::vector<int64_t> res_ids;     // sample index of each resident tree
    int32_t *d_res_par = nullptr;     // [res_count * n] parents
    int64_t *d_res_f = nullptr;       // [res_count] f of each tree on the current graph
    int64_t *d_res_f_alt = nullptr;   // [res_count] where f is recomputed; swapped in on success
    // graph arrays on the device
    int64_t *d_off = nullptr;
    int32_t *d_adj = nullptr, *d_p0 = nullptr, *d_order = nullptr, *d_pre0 = nullptr;
    int32_t *d_out0 = nullptr, *d_eoff = nullptr, *d_elist = nullptr;
    int4 *d_vrec = nullptr;
    int32_t *d_anc0 = nullptr;
    int32_t anc_depth = 0;
    // workspace
    int ws_slots = 0;
    int ws_asked = 0;         // slots the allocation was asked for (the budget may have held fewer)
    bool ws_trav = false, ws_fen = false;
    int64_t ws_fen_len = 0;  // per-slot Fenwick length the buffer was sized for (2m + 2)
    unsigned char *d_state = nullptr;  // per slot: kc::state_bytes(n)
    int4 *d_queue = nullptr;
    int32_t *d_cstart = nullptr;
    int4 *d_rec = nullptr;
    int64_t *d_fen = nullptr;
    int64_t *d_f = nullptr, *d_steps = nullptr, *d_iters = nullptr;  // internal per-sample buffers
    int64_t fbuf_len = 0;
    int32_t *d_ctl = nullptr;
    int64_t *h_progress = nullptr;  // pinned host array, one counter per slot
    int64_t *d_progress = nullptr;  // its device view
    int progress_len = 0;
    kc::ReduceOut *d_red = nullptr;
};

namespace kc_host {

// Record a detail message for kc_last_error() and return st.
kc_status fail(kc_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return kc_host::fail(e_ == hipErrorOutOfMemory ? KC_ERR_NOMEM : KC_ERR_DEVICE, "%s: %s", \
                                 #expr, hipGetErrorString(e_));                                \
    } while (0)

// Device bytes one sample in flight needs: sampler state, plus the numbering
// arrays (trav) and the sweep's Fenwick tree (fen).
int64_t slot_bytes(const kc_graph *g, bool trav, bool fen);
// Samples in flight when the graph's slots option is 0: resident workgroups of the kernel.
int default_slots(const kc_graph *g, bool batch = false);  // resident workgroups of the launch's kernel
int64_t workspace_budget(const kc_graph *g, size_t free_b);
// Slots that split `count` samples into equal waves (at most `slots`).
int balanced_slots(int slots, int64_t count);
// The graph's device arrays as the kernels see them.
kc::GraphDev graph_dev(const kc_graph *g);
// The options of g that every launch carries (walkers, traversal, step cap, status word).
void fill_run_options(const kc_graph *g, kc::RunParams &rp);
// Launch the persistent kernel on a prepared workspace and check the status it reports.
kc_status launch_checked(kc_graph *g, const kc::SlotDev &sd, const kc::RunParams &rp, int slots,
                         hipStream_t stream);
// kappa and its standard error from the exact sums and count already in *res (Theorem 3.3).
void finish_result(int64_t two_m, kc_result *res);
// Exact sums of f (and draws, sampler rounds) over count samples into *res, with kappa
// and its standard error (Theorem 3.3).
kc_status finish_reduce(kc_graph *g, int32_t count, const int64_t *f, const int64_t *steps,
                        const int64_t *iters, kc_result *res, hipStream_t stream);

}  // namespace kc_host
