// kc_internal.h -- structures shared by the library's host code (kc_host.cpp)
// and its kernels (kc_device.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

// Graph arrays resident on the device (read-only during sampling/traversal).
struct GraphDev {
    int32_t n;
    int32_t root;
    int64_t two_m;
    const int64_t *off;   // [n+1] CSR row offsets
    const int32_t *adj;   // [2m]  CSR neighbours, ascending per row
    const int32_t *p0;    // [n]   tau0 parent (-1 at the root)
    const int32_t *order; // [n]   walk start order: BFS order from the root
    const int32_t *pre0;  // [n]   vertex at tau0 preorder position
    const int32_t *out0;  // [n]   last tau0 preorder position inside Sub(tau0, v)
    const int32_t *eoff;  // [nblk+1] per 64-position block: vertices whose tau0
    const int32_t *elist; //          subtree started before the block and ends in it
    const int4 *vrec;     // [2n]  32-byte record per vertex: {offset, degree, first six
                          //       neighbours (-1 past the degree)}
    const int32_t *anc0;  // [anc_depth * n] level-major tau0 ancestors: anc0[i n + v] is the
                          //       (i+1)-th ancestor of v, -1 past the root; null if tau0 is deep
    int32_t anc_depth;    //       levels in anc0 (4 or 8), 0 without the table
};

// Per-slot workspace: one slot = one sample in flight = one wavefront.
//
// A slot's state block (state_bytes(stride) bytes) holds the sampler's arrays:
//   tag words  uint64 [stride] at 0: tag/flag bits | first parked chain + 1 << 32
//   arrow words uint64 [stride] at 8 stride: arrow target | draws << 32
//   restart ring int32 [stride] at 16 stride
// Once the tree's parents are copied into rec they are dead, and the tree
// numbering reuses the block:
//   ord  int4 [stride] at 0: finished vertices {v, parent, vol, offset}, leaves {v, parent, deg, 0}
//   grp  int32 [stride + 1] at 16 stride: completion group boundaries
struct SlotDev {
    unsigned char *state; // [slots * state_bytes(stride)]
    int4 *queue;     // [slots*chains] sampler: ready tasks
    int32_t *cstart; // [slots*chains] sampler: chain start vertices
    int64_t chains;  // per-slot stride of queue and cstart
    int4 *rec;       // [slots*stride] the numbered tree, 16 bytes per vertex: numbering word, then
                     // parent | deg, later parent | tin; null without the traversal
    int64_t *fen;    // [slots*fen_len] Fenwick tree (sweep traversal only)
    int64_t fen_len; // per-slot length of fen: 2m + 2 (0 if not allocated)
    int64_t stride;  // vertices per slot (a batch: its largest graph's n)
};

// Bytes of one slot's state block: 20 bytes per vertex, the 4 of grp's last
// entry, rounded up to 256 so that every slot's block starts 256-aligned.
__host__ __device__ inline int64_t state_bytes(int64_t stride) { return (20 * stride + 4 + 255) / 256 * 256; }

// One graph's share of a batch launch (batch_kernel).
struct BatchJob {
    GraphDev g;
    uint64_t seed;
    int64_t first;      // sample index of the job's first item at launch 0
    int64_t iter_cap;   // sampler rounds per sample
    int32_t walkers, traversal, lean;
};

constexpr int BATCH_MAX = 8;  // graphs in one batch launch

// Kernel arguments of a batch launch: k jobs; job j owns work items
// base[j] .. base[j+1]-1, whose f, draws and rounds go to f/steps/iters[idx].
struct BatchArgs {
    int32_t k;
    int32_t base[BATCH_MAX + 1];
    BatchJob job[BATCH_MAX];
    int64_t *f, *steps, *iters;
};

enum RunMode { RUN_SAMPLE = 0, RUN_ESTIMATE = 1, RUN_EVALUATE = 2, RUN_CURRENT = 3, RUN_CROSS = 4 };

// Counter words 2 and 3 of the Philox draw that picks a link-cut or cut-link
// edge: (tree slot, update number, ISM_CTR_LO, ISM_CTR_HI), a counter no tree
// sample uses.
constexpr uint32_t ISM_CTR_LO = 0xFFFFFFFEu, ISM_CTR_HI = 0xFFFFFFFFu;

struct RunParams {
    uint64_t seed;
    int64_t first;
    int32_t count;
    int32_t walkers;    // 1..64
    int32_t mode;       // RunMode
    int32_t traversal;  // 1 walk, 2 sweep
    int32_t lean;       // 1: a walk's look at its next vertex is the claim alone (results do
                        //    not depend on it)
    int64_t iter_cap;   // sampler iterations per sample
    const int32_t *parents_in; // RUN_EVALUATE input [count*n]
    int32_t *parents_out;      // RUN_SAMPLE  [count*n]
    uint32_t *cnt_out;         // RUN_SAMPLE  [count*n] (optional)
    int64_t *steps_out;        // [count] (optional)
    int64_t *f_out;            // [count] (RUN_ESTIMATE / RUN_EVALUATE)
    int64_t *iters_out;        // [count] sampler rounds per sample (optional)
    int32_t *ctl;              // [4]: work counter, error code, error sample, spare
    int64_t *progress;         // [slots] samples finished per workgroup (host-mapped), or null
    int32_t root_u = -1;       // RUN_SAMPLE: if root_u >= 0, u and v start in the tree instead of
    int32_t root_v = -1;       // the graph's root (a forest of two trees rooted at u and v)
    const int32_t *path = nullptr;  // RUN_CURRENT: vertices of a u -> v path in the graph
    int32_t path_len = 0;           //              number of vertices (>= 2)
    const int32_t *rows = nullptr;  // modes that read parents_in: tree idx is row rows[idx] (null: idx)
    int32_t *parents_mut = nullptr; // RUN_CROSS with relink: the same rows, rewritten in place
    int32_t cut_u = -1, cut_v = -1; // RUN_CROSS: the tree edge whose removal splits the tree
    int32_t relink = 0;             // RUN_CROSS: also re-join by a drawn crossing edge
    uint32_t serial = 0;            // RUN_CROSS: update number of that draw
};

// Device result of the exact reduction.
struct ReduceOut {
    uint64_t sum_lo;
    int64_t sum_hi;
    uint64_t sq_lo;
    uint64_t sq_hi;
    int64_t steps;
    int64_t iters;
    int64_t pad[2];
};

// Error codes written by kernels into ctl[1] (match kc_status values).
enum { DEV_OK = 0, DEV_LIMIT = 6, DEV_PROTOCOL = 8, DEV_BADTREE = 9 };

// Launchers (kc_device.hip).  All are asynchronous on `stream`.
hipError_t launch_reset_ctl(int32_t *ctl, hipStream_t stream);
hipError_t launch_persistent(const GraphDev &g, const SlotDev &s, const RunParams &rp, int chains,
                             int slots, hipStream_t stream);
hipError_t launch_reduce(const int64_t *f, const int64_t *steps, const int64_t *iters, int32_t count,
                         ReduceOut *out, hipStream_t stream);
// A batch: reset of the status word, the persistent launch over every job, the
// exact sums of each job into out[j], and one more on the launch counter.
hipError_t launch_batch(const BatchArgs &a, const SlotDev &s, int32_t *ctl, int64_t *launch, ReduceOut *out,
                        int chains, int slots, hipStream_t stream);
hipError_t launch_zero_i64(int64_t *p, int64_t len, hipStream_t stream);
hipError_t launch_reroot(int32_t *par, int32_t count, int64_t n, int32_t u, int32_t v, int32_t r,
                         hipStream_t stream);
hipError_t launch_link_cut(int32_t *par, const int32_t *rows, int32_t count, int64_t n, int32_t u, int32_t v,
                           uint64_t seed, uint32_t serial, int relink, int64_t *d_out, int32_t *ctl,
                           hipStream_t stream);
hipError_t launch_flag_trees(const int32_t *par, int32_t count, int64_t n, const int32_t *eu,
                             const int32_t *ev, int32_t ne, uint8_t *flags, hipStream_t stream);
bool valid_chains(int chains);            // a built chain-table size?
int persistent_blocks_per_cu(int chains);  // resident workgroups per CU for that size
int batch_blocks_per_cu(int chains);       // the same for the batch kernel
int sampler_chains();                      // queue / chain-start entries to allocate per slot

}  // namespace kc
