// kc_batch.cpp -- batches: one persistent launch over the samples of up to
// eight graphs of any sizes (section 5, Exp-VI runs samples in parallel;
// here samples of different graphs share one launch), captured once as a HIP
// graph and replayed.  Each replay estimates the next block of sample ids of
// every graph; its status and exact sums stay on the device until
// kc_batch_results reads them, so replays need no host round trip.

#include <algorithm>
#include <cstring>

#include "kc_host.h"

using namespace kc_host;

struct kc_batch {
    int32_t k = 0;
    kc_graph *graphs[kc::BATCH_MAX] = {};
    int32_t counts[kc::BATCH_MAX] = {};
    kc::BatchArgs args{};
    kc::SlotDev sd{};
    int slots = 0, chains = 1024;
    int64_t total = 0;
    // device memory owned by the batch
    unsigned char *d_state = nullptr;
    int32_t *d_cstart = nullptr, *d_ctl = nullptr;
    int4 *d_queue = nullptr, *d_rec = nullptr;
    int64_t *d_fen = nullptr, *d_f = nullptr, *d_steps = nullptr, *d_iters = nullptr, *d_launch = nullptr;
    kc::ReduceOut *d_red = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void batch_free(kc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    void *bufs[] = {b->d_state, b->d_cstart, b->d_ctl, b->d_queue, b->d_rec, b->d_fen, b->d_f, b->d_steps,
                    b->d_iters, b->d_launch, b->d_red};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    delete b;
}

template <typename T>
hipError_t alloc_n(T **p, size_t count) {
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
}

}  // namespace

extern "C" {

kc_status kc_batch_create(kc_graph *const *graphs, int32_t k, const uint64_t *seeds, const int64_t *firsts,
                          const int32_t *counts, void *hip_stream, kc_batch **out) {
    if (!out) return fail(KC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (k < 1 || k > kc::BATCH_MAX) return fail(KC_ERR_INVALID, "a batch holds 1..%d graphs (k=%d)", kc::BATCH_MAX, k);
    if (!graphs || !seeds || !firsts || !counts) return fail(KC_ERR_INVALID, "NULL argument");
    int64_t total = 0, max_n = 0, max_fen = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (!graphs[j]) return fail(KC_ERR_INVALID, "graph %d is NULL", j);
        if (counts[j] < 1 || firsts[j] < 0) return fail(KC_ERR_INVALID, "job %d: count must be >= 1, first >= 0", j);
        total += counts[j];
        max_n = std::max(max_n, graphs[j]->n);
        if (graphs[j]->traversal == KC_TRAV_SWEEP) max_fen = std::max(max_fen, graphs[j]->two_m + 2);
    }
    if (total >= (1ll << 31)) return fail(KC_ERR_INVALID, "%lld samples per launch exceed 2^31", (long long)total);
    hipStream_t stream = (hipStream_t)hip_stream;
    kc_batch *b = new (std::nothrow) kc_batch();
    if (!b) return fail(KC_ERR_NOMEM, "host allocation failed");
    b->k = k;
    b->total = total;
    b->chains = graphs[0]->chains;
    kc::BatchArgs &a = b->args;
    a.k = k;
    a.base[0] = 0;
    for (int32_t j = 0; j < k; ++j) {
        kc_graph *g = graphs[j];
        b->graphs[j] = g;
        b->counts[j] = counts[j];
        a.base[j + 1] = a.base[j] + counts[j];
        kc::RunParams rp{};
        fill_run_options(g, rp);
        kc::BatchJob &job = a.job[j];
        job.g = graph_dev(g);
        job.seed = seeds[j];
        job.first = firsts[j];
        job.iter_cap = rp.iter_cap;
        job.walkers = rp.walkers;
        job.traversal = rp.traversal;
        job.lean = rp.lean;
    }
    // samples in flight: the first graph's slots option (else the kernel's resident
    // workgroups), within its memory budget for slots sized for the largest graph
    const size_t n = (size_t)max_n, ch = (size_t)kc::sampler_chains();
    const int64_t per_slot = kc::state_bytes(max_n) + (int64_t)(20 * ch + 16 * n + 8 * (size_t)max_fen);
    int want = graphs[0]->slots_opt > 0 ? graphs[0]->slots_opt : default_slots(graphs[0], true);
    want = (int)std::min<int64_t>(want, total);
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(KC_ERR_DEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
    }
    const int64_t budget = workspace_budget(graphs[0], free_b);
    int slots = (int)std::min<int64_t>(want, budget / per_slot);
    slots = balanced_slots(slots, total);
    if (slots < 1) {
        batch_free(b);
        return fail(KC_ERR_NOMEM, "one sample of the largest graph needs %lld bytes of workspace, budget %lld",
                    (long long)per_slot, (long long)budget);
    }
    b->slots = slots;
    const size_t S = (size_t)slots;
    e = alloc_n(&b->d_state, S * (size_t)kc::state_bytes(max_n));
    if (e == hipSuccess) e = alloc_n(&b->d_queue, S * ch);
    if (e == hipSuccess) e = alloc_n(&b->d_cstart, S * ch);
    if (e == hipSuccess) e = alloc_n(&b->d_rec, S * n);
    if (e == hipSuccess && max_fen > 0) e = alloc_n(&b->d_fen, S * (size_t)max_fen);
    if (e == hipSuccess) e = alloc_n(&b->d_f, (size_t)total);
    if (e == hipSuccess) e = alloc_n(&b->d_steps, (size_t)total);
    if (e == hipSuccess) e = alloc_n(&b->d_iters, (size_t)total);
    if (e == hipSuccess) e = alloc_n(&b->d_ctl, 4);
    if (e == hipSuccess) e = alloc_n(&b->d_launch, 1);
    if (e == hipSuccess) e = alloc_n(&b->d_red, (size_t)k);
    // the Fenwick trees and the launch counter start at zero (fill kernels, outside the capture)
    if (e == hipSuccess && max_fen > 0) e = kc::launch_zero_i64(b->d_fen, (int64_t)S * max_fen, stream);
    if (e == hipSuccess) e = kc::launch_zero_i64(b->d_launch, 1, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(e == hipErrorOutOfMemory ? KC_ERR_NOMEM : KC_ERR_DEVICE, "batch set-up: %s", hipGetErrorString(e));
    }
    kc::SlotDev &sd = b->sd;
    sd.state = b->d_state;
    sd.queue = b->d_queue;
    sd.cstart = b->d_cstart;
    sd.chains = (int64_t)ch;
    sd.rec = b->d_rec;
    sd.fen = b->d_fen;
    sd.fen_len = max_fen;
    sd.stride = max_n;
    a.f = b->d_f;
    a.steps = b->d_steps;
    a.iters = b->d_iters;
    // capture the launch sequence once on a stream of the batch's own
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e1 = kc::launch_batch(a, sd, b->d_ctl, b->d_launch, b->d_red, b->chains, slots, b->cap);
        const hipError_t e2 = hipStreamEndCapture(b->cap, &b->graph);
        e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(KC_ERR_DEVICE, "capturing the batch launch: %s", hipGetErrorString(e));
    }
    *out = b;
    return KC_OK;
}

kc_status kc_batch_launch(kc_batch *b, void *hip_stream) {
    if (!b) return fail(KC_ERR_INVALID, "NULL batch");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
    return KC_OK;
}

kc_status kc_batch_results(kc_batch *b, kc_result *results, int64_t *launches, void *hip_stream) {
    if (!b || !results) return fail(KC_ERR_INVALID, "NULL argument");
    hipStream_t stream = (hipStream_t)hip_stream;
    int32_t ctl[4] = {0, 0, 0, 0};
    kc::ReduceOut red[kc::BATCH_MAX];
    int64_t nl = 0;
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(ctl, b->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(red, b->d_red, sizeof(kc::ReduceOut) * (size_t)b->k, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&nl, b->d_launch, sizeof(nl), hipMemcpyDeviceToHost));
    if (launches) *launches = nl;
    if (ctl[1] != 0) {
        int j = 0;
        while (j + 1 < b->k && ctl[2] >= b->args.base[j + 1]) ++j;
        const long long s = (long long)(b->args.job[j].first + (nl - 1) * b->counts[j] + (ctl[2] - b->args.base[j]));
        if (ctl[1] == kc::DEV_LIMIT) return fail(KC_ERR_LIMIT, "graph %d, sample %lld exceeded the step limit", j, s);
        return fail(KC_ERR_DEVICE, "sampler protocol violation (code %d) in graph %d, sample %lld", ctl[1], j, s);
    }
    for (int32_t j = 0; j < b->k; ++j) {
        kc_result &r = results[j];
        r = kc_result{};
        r.sum_f_lo = red[j].sum_lo;
        r.sum_f_hi = red[j].sum_hi;
        r.sum_f2_lo = red[j].sq_lo;
        r.sum_f2_hi = red[j].sq_hi;
        r.count = b->counts[j];
        r.total_steps = red[j].steps;
        r.sampler_iterations = red[j].iters;
        finish_result(b->graphs[j]->two_m, &r);
    }
    return KC_OK;
}

kc_status kc_batch_f(const kc_batch *b, int32_t j, int64_t *f_out, void *hip_stream) {
    if (!b || !f_out) return fail(KC_ERR_INVALID, "NULL argument");
    if (j < 0 || j >= b->k) return fail(KC_ERR_INVALID, "graph %d is not in the batch", j);
    HIP_TRY(hipMemcpyAsync(f_out, b->d_f + b->args.base[j], sizeof(int64_t) * (size_t)b->counts[j],
                           hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    return KC_OK;
}

kc_status kc_batch_destroy(kc_batch *b) {
    if (b) batch_free(b);
    return KC_OK;
}

}  // extern "C"
