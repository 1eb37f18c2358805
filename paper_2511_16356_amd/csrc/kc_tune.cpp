// kc_tune.cpp -- kc_autotune: chooses a graph's launch options (samples in
// flight, chain-table size, walkers per sample, traversal) by timing short estimates, and keeps the choice in a cache file.
// None of these options changes any tree, f or estimate: the tree of sample s
// is the cycle-popping outcome of its arrows (section 2.2) whatever the launch
// shape, and f is Theorem 3.4's sum whatever the traversal.
//
// Cache: one JSON object per line,
//   {"key": "<arch>|n=..|two_m=..|dmax=..|depth0=..|count=..", "chains": C, "slots": S,
//    "walkers": W, "traversal": T, "samples_per_s": R}
// The last line with the graph's key wins.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "kc_host.h"

using namespace kc_host;

namespace {

struct Choice {
    int32_t chains, slots, walkers, traversal;
};

std::string cache_key(const kc_graph *g, int32_t count) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|n=%lld|two_m=%lld|dmax=%d|depth0=%d|count=%d", arch.c_str(), (long long)g->n,
                  (long long)g->two_m, g->max_degree, g->depth0, count);
    return buf;
}

// The integer after "\"name\":" in a cache line (or fallback).
long long field(const std::string &line, const char *name, long long fallback) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return fallback;
    return std::strtoll(line.c_str() + p + pat.size(), nullptr, 10);
}

bool cache_lookup(const char *path, const std::string &key, Choice *c) {
    FILE *fh = path ? std::fopen(path, "r") : nullptr;
    if (!fh) return false;
    const std::string want = "\"key\": \"" + key + "\"";
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof(line), fh)) {
        const std::string l(line);
        if (l.find(want) == std::string::npos) continue;
        c->chains = (int32_t)field(l, "chains", 1024);
        c->slots = (int32_t)field(l, "slots", 0);
        c->walkers = (int32_t)field(l, "walkers", 64);
        c->traversal = (int32_t)field(l, "traversal", KC_TRAV_AUTO);
        found = true;
    }
    std::fclose(fh);
    return found;
}

void cache_store(const char *path, const std::string &key, const Choice &c, double rate) {
    FILE *fh = path ? std::fopen(path, "a") : nullptr;
    if (!fh) return;
    std::fprintf(fh,
                 "{\"key\": \"%s\", \"chains\": %d, \"slots\": %d, \"walkers\": %d, \"traversal\": %d, "
                 "\"samples_per_s\": %.3f}\n",
                 key.c_str(), c.chains, c.slots, c.walkers, c.traversal, rate);
    std::fclose(fh);
}

kc_status apply(kc_graph *g, const Choice &c) {
    kc_status st = kc_set_option(g, KC_OPT_CHAINS, c.chains);
    if (st == KC_OK) st = kc_set_option(g, KC_OPT_SLOTS, c.slots);
    if (st == KC_OK) st = kc_set_option(g, KC_OPT_WALKERS, c.walkers);
    if (st == KC_OK) st = kc_set_option(g, KC_OPT_TRAVERSAL, c.traversal);
    return st;
}

}  // namespace

extern "C" kc_status kc_autotune(kc_graph *g, int32_t count, const char *cache_path, kc_tune_result *out,
                                 void *hip_stream) {
    if (!g || !out) return fail(KC_ERR_INVALID, "NULL argument");
    if (count < 1) return fail(KC_ERR_INVALID, "count must be >= 1");
    std::memset(out, 0, sizeof(*out));
    const std::string key = cache_key(g, count);
    Choice best{};
    if (cache_lookup(cache_path, key, &best)) {
        const kc_status st = apply(g, best);
        if (st != KC_OK) return st;
        out->chains = best.chains;
        out->slots = best.slots;
        out->walkers = best.walkers;
        out->traversal = best.traversal;
        out->from_cache = 1;
        return KC_OK;
    }
    const Choice start{g->chains, g->slots_opt, g->walkers, g->trav_opt};
    // samples in flight by default: the kernel's resident workgroups, as many as fit the
    // memory budget (measured with the graph's own workspace freed first)
    kc_status st = kc_trim(g, hip_stream);
    if (st != KC_OK) return st;
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const int64_t budget = workspace_budget(g, free_b);
    const int64_t fit = budget / std::max<int64_t>(1, slot_bytes(g, true, g->traversal == KC_TRAV_SWEEP));
    const int full = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(default_slots(g), count), fit));
    // trial estimates: one wave of samples in flight (at least 64), on sample ids far
    // from any the caller uses (2^40 upward)
    kc_result res{};
    int64_t next_first = 1ll << 40;
    auto trial = [&](const Choice &c, double *rate) -> kc_status {
        kc_status st = apply(g, c);
        if (st != KC_OK) return st;
        const int slots = c.slots > 0 ? c.slots : full;
        const int32_t t = (int32_t)std::min<int64_t>(count, std::max<int64_t>(64, slots));
        st = kc_reserve(g, t, hip_stream);
        if (st != KC_OK) return st;
        const auto t0 = std::chrono::steady_clock::now();
        st = kc_estimate(g, 0, next_first, t, &res, nullptr, nullptr, hip_stream);
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        next_first += t;
        if (st != KC_OK) return st;
        *rate = (double)t / std::max(dt, 1e-9);
        out->trials += 1;
        return KC_OK;
    };
    best = start;
    double best_rate = 0.0;
    st = trial(best, &best_rate);
    if (st != KC_OK) {
        (void)apply(g, start);
        return st;
    }
    out->start_samples_per_s = best_rate;
    // one dimension at a time, each candidate a change of the best choice so far
    using Change = std::function<void(Choice &)>;
    std::vector<Change> changes;
    if (g->depth0 <= 64) {  // the walk costs n * depth0 per tree: only shallow reference trees try both
        changes.push_back([](Choice &c) { c.traversal = KC_TRAV_WALK; });
        changes.push_back([](Choice &c) { c.traversal = KC_TRAV_SWEEP; });
    }
    changes.push_back([](Choice &c) { c.chains = c.chains == 1024 ? 2048 : 1024; });
    changes.push_back([full](Choice &c) { c.slots = std::max(1, full * 3 / 4); });
    changes.push_back([full](Choice &c) { c.slots = std::max(1, full / 2); });
    changes.push_back([](Choice &c) { c.walkers = c.walkers == 64 ? 32 : 64; });
    for (const Change &change : changes) {
        Choice cand = best;
        change(cand);
        if (std::memcmp(&cand, &best, sizeof(Choice)) == 0) continue;
        double rate = 0.0;
        st = trial(cand, &rate);
        if (st == KC_ERR_NOMEM) continue;  // a shape that does not fit is skipped
        if (st != KC_OK) {
            (void)apply(g, start);
            return st;
        }
        if (rate > best_rate * 1.02) {  // keep a change only for a clear gain
            best = cand;
            best_rate = rate;
        }
    }
    st = apply(g, best);
    if (st != KC_OK) return st;
    cache_store(cache_path, key, best, best_rate);
    out->chains = best.chains;
    out->slots = best.slots;
    out->walkers = best.walkers;
    out->traversal = best.traversal;
    out->samples_per_s = best_rate;
    return KC_OK;
}
