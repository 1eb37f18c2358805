// kc_static.hip -- kc_estimate_static: the estimate of kc_estimate with every
// byte of workspace taken from one static device array instead of allocated
// memory, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is held by every device the library runs on
// until the process ends.  Host code never passes its name to a kernel: the
// name is a host-side stand-in, not a device address.  Its device address is
// looked up once per device, with that device current, by
// hipGetSymbolAddress, and only that address is used afterwards.  Every call
// on one device shares the device's array and leaves the last call's contents
// behind; calls that overlap on one device race.

#include <mutex>

#include "kc_host.h"

namespace {

// Bytes of the static workspace on each device.
constexpr size_t STATIC_SCRATCH_BYTES = 256ull << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up on the
// first call on that device.
hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Carves consecutive 256-byte-aligned regions out of [base, base + cap).
struct Carver {
    unsigned char *base;
    size_t cap, used = 0;
    template <typename T>
    T *take(size_t count) {
        const size_t off = (used + 255) & ~(size_t)255;
        const size_t bytes = count * sizeof(T);
        if (off + bytes > cap) return nullptr;
        used = off + bytes;
        return reinterpret_cast<T *>(base + off);
    }
};

}  // namespace

extern "C" kc_status kc_estimate_static(kc_graph *g, uint64_t seed, int64_t first_sample, int32_t count,
                                        kc_result *result, int64_t *f_out, void *hip_stream) {
    using namespace kc_host;
    if (!g || !result) return fail(KC_ERR_INVALID, "NULL graph or result");
    if (count < 1 || first_sample < 0) return fail(KC_ERR_INVALID, "count must be >= 1");
    hipStream_t stream = (hipStream_t)hip_stream;
    void *base = nullptr;
    HIP_TRY(scratch_address(&base));
    const bool fen = g->traversal == KC_TRAV_SWEEP;
    const size_t n = (size_t)g->n;
    const size_t chains = (size_t)kc::sampler_chains();
    // per-sample results first, then as many slots as fit
    Carver c{static_cast<unsigned char *>(base), STATIC_SCRATCH_BYTES};
    int64_t *f = f_out ? f_out : c.take<int64_t>((size_t)count);
    int64_t *steps = c.take<int64_t>((size_t)count);
    int64_t *iters = c.take<int64_t>((size_t)count);
    if (!f || !steps || !iters)
        return fail(KC_ERR_NOMEM, "%d samples need %zu bytes of per-sample results; the static workspace holds %zu",
                    count, (size_t)count * (f_out ? 16 : 24), STATIC_SCRATCH_BYTES);
    // bytes of the slot arrays for s samples in flight, each array starting on 256 bytes
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    auto need = [&](size_t s) {
        return r256(s * (size_t)kc::state_bytes(g->n)) + r256(16 * s * chains) + r256(4 * s * chains) +
               r256(16 * s * n) + (fen ? r256(8 * s * (size_t)(g->two_m + 2)) : 0);
    };
    const size_t room = STATIC_SCRATCH_BYTES - r256(c.used);
    int slots = g->slots_opt > 0 ? g->slots_opt : default_slots(g);
    slots = std::min(slots, count);
    while (slots > 0 && need((size_t)slots) > room) slots = (int)std::min<size_t>(slots - 1, room / need(1));
    if (slots < 1)
        return fail(KC_ERR_NOMEM, "one sample in flight needs %zu bytes of workspace; %zu of the %zu-byte static "
                    "workspace are left after the per-sample results", need(1), room, STATIC_SCRATCH_BYTES);
    slots = balanced_slots(slots, count);
    kc::SlotDev sd;
    sd.state = c.take<unsigned char>((size_t)slots * (size_t)kc::state_bytes(g->n));
    sd.queue = c.take<int4>((size_t)slots * chains);
    sd.cstart = c.take<int32_t>((size_t)slots * chains);
    sd.chains = (int64_t)chains;
    sd.rec = c.take<int4>((size_t)slots * n);
    sd.stride = g->n;
    sd.fen = fen ? c.take<int64_t>((size_t)slots * (size_t)(g->two_m + 2)) : nullptr;
    sd.fen_len = fen ? g->two_m + 2 : 0;
    if (!sd.state || !sd.queue || !sd.cstart || !sd.rec || (fen && !sd.fen))
        return fail(KC_ERR_DEVICE, "static workspace layout overflow (%d slots of %zu bytes)", slots, need(1));
    // the sweep's Fenwick trees must start at zero; an earlier call may have left anything
    if (fen) HIP_TRY(kc::launch_zero_i64(sd.fen, (int64_t)slots * sd.fen_len, stream));
    kc::RunParams rp{};
    rp.seed = seed;
    rp.first = first_sample;
    rp.count = count;
    rp.mode = kc::RUN_ESTIMATE;
    rp.f_out = f;
    rp.steps_out = steps;
    rp.iters_out = iters;
    rp.progress = nullptr;
    fill_run_options(g, rp);
    kc_status st = launch_checked(g, sd, rp, slots, stream);
    if (st != KC_OK) return st;
    return finish_reduce(g, count, f, steps, iters, result, stream);
}
