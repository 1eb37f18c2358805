/*
 * kc_probe.h -- C ABI of libkc_probe.so: measured memory ceilings of the
 * current HIP device, used to read the estimator's HBM roofline.  Not part of
 * the estimator (the Wilson draws of Algorithm 1 each touch one random 64-byte
 * line of per-sample state; these calls measure how fast the device serves
 * such lines, and a streaming read for comparison).
 *
 * Both calls run on the null stream, time one launch after a warm-up launch
 * with HIP events, and return 0 on success or a negative code (bad argument,
 * HIP error).  `buf` is a DEVICE pointer the caller owns (contents arbitrary,
 * read only); `sink` is a DEVICE pointer to one int64 that the kernels may
 * write (so that the reads are not optimised away).
 */
#ifndef KC_PROBE_H
#define KC_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming read of `bytes` bytes (16-byte loads, grid-stride); *gbps
 * receives bytes / time in GB/s (10^9 bytes per second). */
int kc_probe_stream_read(const void *buf, size_t bytes, int64_t *sink, double *gbps);

/* About `reads` independent reads of whole 64-byte lines at pseudo-random
 * line indices in [0, bytes / 64) (16 per thread); *sectors_per_s receives
 * lines read per second. */
int kc_probe_random_read(const void *buf, size_t bytes, int64_t reads, int64_t *sink, double *sectors_per_s);

/* Streaming read with `inflight` (1, 2, 4 or 8) 16-byte loads in flight per
 * thread and `blocks_per_cu` (1..64) 256-thread blocks per compute unit;
 * *gbps receives bytes / time in GB/s. */
int kc_probe_stream_sweep(const void *buf, size_t bytes, int inflight, int blocks_per_cu, int64_t *sink,
                          double *gbps);

/* Random line reads in the estimator's shapes, for a sweep of the settings:
 *   shape    : 0 = each lane reads 8 bytes of its own random 64-byte line,
 *              1 = 16 bytes of its own line, 2 = four lanes read one line's
 *              four 16-byte quarters
 *   inflight : reads each thread keeps in flight (1, 2, 4, 8, 16 or 32)
 *   blocks_per_cu : 256-thread blocks per compute unit (1..64)
 * About 2^28 line reads per launch; *lines_per_s receives distinct 64-byte
 * lines read per second. */
int kc_probe_random_sweep(const void *buf, size_t bytes, int shape, int inflight, int blocks_per_cu,
                          int64_t *sink, double *lines_per_s);

#ifdef __cplusplus
}
#endif

#endif /* KC_PROBE_H */
