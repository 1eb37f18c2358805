// kc_probe.hip -- measured memory ceilings of the device, for reading the
// estimator's roofline: a streaming read of a large buffer, and independent
// random reads of 64-byte lines from it (the access pattern of a Wilson draw
// touching a vertex's per-sample state).  Not part of the estimator.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/kc_probe.h"

namespace {

constexpr int BLOCK = 256;

__global__ void __launch_bounds__(BLOCK) stream_read_kernel(const int4 *buf, size_t n16, int64_t *sink) {
    int64_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n16; i += (size_t)gridDim.x * BLOCK) {
        const int4 v = buf[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x7fffffffffffll) sink[0] = acc;  // keeps the loads; never true for the filled buffer
}

// Each thread reads `per_thread` 64-byte lines at indices from a 64-bit mix of
// (thread, k): all reads of a thread are independent, so the memory system
// sees as many lines in flight as it can hold.
__global__ void __launch_bounds__(BLOCK) random_read_kernel(const int4 *buf, size_t lines, int per_thread,
                                                             int64_t *sink) {
    const uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    int64_t acc = 0;
#pragma unroll 4
    for (int k = 0; k < per_thread; ++k) {
        uint64_t h = (t * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)k * 0xC2B2AE3D27D4EB4Full);
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        const size_t line = (size_t)(h % lines);
        const int4 *p = buf + line * 4;
        const int4 a = p[0], b = p[1], c = p[2], d = p[3];
        acc += (a.x ^ b.y) + (c.z ^ d.w);
    }
    if (acc == 0x7fffffffffffll) sink[0] = acc;
}

// Streaming read with K 16-byte loads in flight per thread and round.
template <int K>
__global__ void __launch_bounds__(BLOCK) stream_sweep_kernel(const int4 *buf, size_t n16, int64_t *sink) {
    int64_t acc = 0;
    const size_t stride = (size_t)gridDim.x * BLOCK;
    for (size_t base = (size_t)blockIdx.x * BLOCK + threadIdx.x; base < n16; base += stride * K) {
        int4 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = base + (size_t)k * stride;
            v[k] = i < n16 ? buf[i] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) acc += v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
    }
    if (acc == 0x7fffffffffffll) sink[0] = acc;
}

// Random reads in the shapes the estimator issues: every lane reads W bytes
// (8 or 16) from its own pseudo-random 64-byte line, or (Q = 4) four lanes read
// the four 16-byte quarters of one line; each thread keeps K reads in flight
// (all K addresses are formed and issued before any result is used).
__device__ __forceinline__ uint64_t mix(uint64_t t, uint64_t k) {
    uint64_t h = (t * 0x9E3779B97F4A7C15ull) ^ (k * 0xC2B2AE3D27D4EB4Full);
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    return h;
}

template <int W, int Q, int K>
__global__ void __launch_bounds__(BLOCK) random_sweep_kernel(const unsigned char *buf, size_t lines, int rounds,
                                                             int64_t *sink) {
    const uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    const uint64_t line_owner = t / Q;  // Q lanes share one line
    const int quarter = (int)(t % Q);
    int64_t acc = 0;
    for (int r = 0; r < rounds; ++r) {
        size_t off[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t line = (size_t)(mix(line_owner, (uint64_t)(r * K + k)) % lines);
            off[k] = line * 64 + (size_t)quarter * 16;
        }
        if (W == 8) {
            int64_t v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = *reinterpret_cast<const int64_t *>(buf + off[k]);
#pragma unroll
            for (int k = 0; k < K; ++k) acc += v[k];
        } else {
            int4 v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = *reinterpret_cast<const int4 *>(buf + off[k]);
#pragma unroll
            for (int k = 0; k < K; ++k) acc += v[k].x ^ v[k].w;
        }
    }
    if (acc == 0x7fffffffffffll) sink[0] = acc;
}

int time_launch(void (*launch)(void *), void *arg, double *ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    launch(arg);  // warm-up
    bool ok = hipEventRecord(e0, nullptr) == hipSuccess;
    launch(arg);
    ok = ok && hipEventRecord(e1, nullptr) == hipSuccess;
    ok = ok && hipEventSynchronize(e1) == hipSuccess;
    float f = 0.f;
    ok = ok && hipEventElapsedTime(&f, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return ok && hipGetLastError() == hipSuccess ? 0 : -3;
}

struct StreamArgs { const int4 *buf; size_t n16; int64_t *sink; int blocks; };
struct RandomArgs { const int4 *buf; size_t lines; int per_thread; int64_t *sink; int blocks; };

void launch_stream(void *p) {
    const StreamArgs *a = static_cast<const StreamArgs *>(p);
    hipLaunchKernelGGL(stream_read_kernel, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->n16, a->sink);
}
void launch_random(void *p) {
    const RandomArgs *a = static_cast<const RandomArgs *>(p);
    hipLaunchKernelGGL(random_read_kernel, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->lines,
                       a->per_thread, a->sink);
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

struct SweepArgs { const unsigned char *buf; size_t lines; int rounds; int64_t *sink; int blocks; int shape; int inflight; };

template <int W, int Q, int K>
void launch_sweep_k(const SweepArgs *a) {
    hipLaunchKernelGGL((random_sweep_kernel<W, Q, K>), dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->lines,
                       a->rounds, a->sink);
}

template <int W, int Q>
void launch_sweep_shape(const SweepArgs *a) {
    switch (a->inflight) {
        case 1: launch_sweep_k<W, Q, 1>(a); break;
        case 2: launch_sweep_k<W, Q, 2>(a); break;
        case 4: launch_sweep_k<W, Q, 4>(a); break;
        case 8: launch_sweep_k<W, Q, 8>(a); break;
        case 16: launch_sweep_k<W, Q, 16>(a); break;
        default: launch_sweep_k<W, Q, 32>(a); break;
    }
}

struct StreamSweepArgs { const int4 *buf; size_t n16; int64_t *sink; int blocks; int inflight; };

void launch_stream_sweep(void *p) {
    const StreamSweepArgs *a = static_cast<const StreamSweepArgs *>(p);
    switch (a->inflight) {
        case 1: hipLaunchKernelGGL(stream_sweep_kernel<1>, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->n16, a->sink); break;
        case 2: hipLaunchKernelGGL(stream_sweep_kernel<2>, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->n16, a->sink); break;
        case 4: hipLaunchKernelGGL(stream_sweep_kernel<4>, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->n16, a->sink); break;
        default: hipLaunchKernelGGL(stream_sweep_kernel<8>, dim3(a->blocks), dim3(BLOCK), 0, nullptr, a->buf, a->n16, a->sink); break;
    }
}

void launch_sweep(void *p) {
    const SweepArgs *a = static_cast<const SweepArgs *>(p);
    if (a->shape == 0) launch_sweep_shape<8, 1>(a);
    else if (a->shape == 1) launch_sweep_shape<16, 1>(a);
    else launch_sweep_shape<16, 4>(a);
}

}  // namespace

extern "C" {

int kc_probe_stream_sweep(const void *buf, size_t bytes, int inflight, int blocks_per_cu, int64_t *sink,
                          double *gbps) {
    if (!buf || !sink || !gbps || bytes < 16 || blocks_per_cu < 1 || blocks_per_cu > 64) return -4;
    if (inflight != 1 && inflight != 2 && inflight != 4 && inflight != 8) return -4;
    StreamSweepArgs a{static_cast<const int4 *>(buf), bytes / 16, sink, device_cus() * blocks_per_cu, inflight};
    double ms = 0.0;
    const int rc = time_launch(launch_stream_sweep, &a, &ms);
    if (rc != 0) return rc;
    *gbps = (double)(a.n16 * 16) / (ms * 1e-3) / 1e9;
    return 0;
}

int kc_probe_random_sweep(const void *buf, size_t bytes, int shape, int inflight, int blocks_per_cu,
                          int64_t *sink, double *lines_per_s) {
    if (!buf || !sink || !lines_per_s || bytes < 64 || shape < 0 || shape > 2 || blocks_per_cu < 1 ||
        blocks_per_cu > 64)
        return -4;
    if (inflight != 1 && inflight != 2 && inflight != 4 && inflight != 8 && inflight != 16 && inflight != 32)
        return -4;
    const int blocks = device_cus() * blocks_per_cu;
    const int q = shape == 2 ? 4 : 1;
    // about 2^28 line reads per launch
    const int64_t threads = (int64_t)blocks * BLOCK;
    int rounds = (int)std::max<int64_t>(1, ((int64_t)1 << 28) * q / (threads * inflight));
    SweepArgs a{static_cast<const unsigned char *>(buf), bytes / 64, rounds, sink, blocks, shape, inflight};
    double ms = 0.0;
    const int rc = time_launch(launch_sweep, &a, &ms);
    if (rc != 0) return rc;
    *lines_per_s = (double)threads / q * rounds * inflight / (ms * 1e-3);
    return 0;
}


int kc_probe_stream_read(const void *buf, size_t bytes, int64_t *sink, double *gbps) {
    if (!buf || !sink || !gbps || bytes < 16) return -4;
    StreamArgs a{static_cast<const int4 *>(buf), bytes / 16, sink, device_cus() * 16};
    double ms = 0.0;
    const int rc = time_launch(launch_stream, &a, &ms);
    if (rc != 0) return rc;
    *gbps = (double)(a.n16 * 16) / (ms * 1e-3) / 1e9;
    return 0;
}

int kc_probe_random_read(const void *buf, size_t bytes, int64_t reads, int64_t *sink, double *sectors_per_s) {
    if (!buf || !sink || !sectors_per_s || bytes < 64 || reads < 1) return -4;
    const int per_thread = 16;
    const int64_t threads = (reads + per_thread - 1) / per_thread;
    const int64_t blocks = (threads + BLOCK - 1) / BLOCK;
    if (blocks > (1ll << 30)) return -4;
    RandomArgs a{static_cast<const int4 *>(buf), bytes / 64, per_thread, sink, (int)blocks};
    double ms = 0.0;
    const int rc = time_launch(launch_random, &a, &ms);
    if (rc != 0) return rc;
    *sectors_per_s = (double)(blocks * BLOCK * per_thread) / (ms * 1e-3);
    return 0;
}

}  // extern "C"
