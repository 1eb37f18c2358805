// kc_device.hip -- gfx950 kernels of the Kemeny-constant estimator.
//
// One wavefront (64 lanes, one workgroup) owns one sample at a time and runs
// its whole hot path in a persistent loop:
//
//   1. Uniform spanning tree by Wilson's algorithm (paper section 2.2 and
//      Algorithm 1), organised as cooperative cycle popping: up to 64 lanes
//      drive loop-erased walks ("chains") of the same sample at once; a chain
//      whose arrow lands on another chain's path is parked in an LDS table
//      and its lane moves on.  The k-th draw at vertex v of sample s always
//      uses the same Philox4x32-10 arrow, so the tree and the per-vertex draw
//      counts are the unique cycle-popping outcome of those arrow stacks,
//      whatever order the pops happen in.
//   2. Subtree volumes vol(v) of the sampled tree (Algorithm 1, the loop that
//      fills vol[]) by bottom-up carriers with one 64-bit atomic per vertex,
//      and a volume-weighted preorder numbering tin(v) of the tree (top-down,
//      replaying the bottom-up completion groups in reverse).  A vertex u lies
//      in Sub(tau, v) iff tin(v) <= tin(u) < tin(v) + vol(v).
//   3. f(tau) of Theorem 3.3 via Theorem 3.4: every tree edge (v, p(v)) that
//      is also a tau0 edge contributes +-(2m - vol(v)) to every u in the
//      intersection of a tau subtree and a tau0 subtree.  Two evaluations:
//        walk  -- per u, walk u's tau0 ancestors (depth0 steps);
//        sweep -- visit tau0 in preorder, 64 positions per step, keeping the
//                 active tau0 ancestors' contributions as range updates in a
//                 Fenwick tree indexed by tin (O(log m) per update/query).
//   4. Exact reduction: sum f and sum f^2 in 128-bit integers.
//
// Cross-lane communication through global memory uses workgroup-scope
// relaxed atomics (L2-coherent on gfx950) ordered by workgroup fences; every
// lane of a sample is in the same wavefront.

#include "kc_internal.h"

namespace kc {
namespace {

constexpr int WAVE = 64;

// ------------------------------------------------------------ memory helpers

template <typename T>
__device__ __forceinline__ T aload(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void astore(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T afetch_add(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T afetch_and(T *p, T v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T afetch_xor(T *p, T v) {
    return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T acas(T *p, T expected, T desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return expected;  // value found at *p
}
__device__ __forceinline__ void fence_wg() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

// ------------------------------------------------------------- wave helpers

__device__ __forceinline__ int rank_in(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ void report_error(int32_t *ctl, int code, int idx) {
    if (threadIdx.x == 0) {
        int expected = 0;
        if (__hip_atomic_compare_exchange_strong(&ctl[1], &expected, code, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_store(&ctl[2], idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ arrows

// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of two 32x32->64 multiplies with the Weyl key schedule.  Counter
// (k, v, s_lo, s_hi), key (seed_lo, seed_hi).  The neighbour slot is the
// high word of x * deg with x = out0 | out1 << 32, i.e. floor(x deg / 2^64),
// computed from two 32x32 products.
struct Bits {
    uint32_t lo, hi;
};
__device__ __forceinline__ Bits philox_bits(uint64_t seed, uint64_t s, uint32_t v, uint32_t k) {
    uint32_t x0 = k, x1 = v, x2 = (uint32_t)s, x3 = (uint32_t)(s >> 32);
    uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one full 32x32->64 product each (a single v_mad_u64_u32, not mul_lo + mul_hi)
        const uint64_t a = (uint64_t)0xD2511F53u * x0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ key0;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ key1;
        x0 = y0; x1 = (uint32_t)b; x2 = y2; x3 = (uint32_t)a;
        key0 += 0x9E3779B9u;
        key1 += 0xBB67AE85u;
    }
    return Bits{x0, x1};
}
__device__ __forceinline__ uint32_t slot_of(Bits x, uint32_t deg) {
    const uint64_t lowprod = (uint64_t)x.lo * deg;
    const uint64_t highprod = (uint64_t)x.hi * deg + (lowprod >> 32);
    return (uint32_t)(highprod >> 32);
}
__device__ __forceinline__ uint32_t arrow_slot(uint64_t seed, uint64_t s, uint32_t v, uint32_t k,
                                               uint32_t deg) {
    return slot_of(philox_bits(seed, s, v, k), deg);
}

// ------------------------------------------------------------ sampler state

// Neighbours kept inline in a vertex's 32-byte graph record (see GraphDev::vrec).
constexpr int VREC_INLINE = 6;
//
// Two 8-byte words per (sample, vertex), in two arrays, so that the claim
// (an atomic on the tag word) and the read of the arrow word go to different
// cache lines and overlap:
//   tag word   low half: bits 0..30 tag (0 = arrow not revealed ("free"),
//              1 = in the tree from the start, 2 + c + CH g = on the path of
//              chain c in its generation g); bit 31 need (the vertex's turn as
//              a walk start passed while it was on a path)
//              high half: 1 + the first of the chains parked on this vertex
//              (their head's arrow points here), 0 if none; the list continues
//              through the chain table's wnext links
//   arrow word low half: the current arrow target (the tree parent at the
//              end); high half: how many arrows the vertex has drawn
// A free vertex's tag word is 0; a start vertex's is T_TREE.  A path that
// reaches the tree joins it as a whole: its chain records the generation as
// finished (fin in LDS), and every vertex tagged with a finished generation is
// a tree vertex from then on, with no write to its tag word.  Every change of
// a tag word is one atomic operation, so claims, parks, need marks and erases
// of the same round may meet on a vertex in any order.
constexpr uint32_t T_FREE = 0, T_TREE = 1, T_CHAIN0 = 2;

__device__ __forceinline__ uint32_t *tag_high(uint64_t *w) { return reinterpret_cast<uint32_t *>(w) + 1; }
__device__ __forceinline__ uint64_t arrow_of(int32_t nxt, uint32_t drw) {
    return (uint64_t)(uint32_t)nxt | ((uint64_t)drw << 32);
}
constexpr uint32_t TW_TAG = (1u << 31) - 1;
constexpr uint32_t TW_NEED = 1u << 31;
constexpr int GEN_MAX = 32767;  // generations of one chain id (fin is int16)

// A chain is a loop-erased path of revealed arrows owned by one walk: from
// its start vertex to its head.  A lane drives at most one chain at a time.
// When the head's arrow lands on another chain's path, the chain is parked
// (it joins the vertex's waiter list) and the lane takes other work; the chain is
// woken when that vertex is popped (resume there), and joins the tree with
// the chain it waits on.  A start vertex that already lies on a path is skipped with its
// need bit set; if it is popped later its eraser queues it for a restart.
// Popped vertices are also offered as optional extra starts (a small LIFO):
// revealing any free vertex is work the cycle-popping order fixes anyway.
// Chain-table sizes the kernel is built for (chains per sample).  More chains
// let more walks proceed at once in one sample (fewer rounds per sample);
// fewer chains let more samples share a CU (more samples in flight).
#define KC_CHAIN_VARIANTS(X) X(1024) X(2048)
constexpr int MAX_CHAINS = 2048;
constexpr int HINTS = 128; // optional restart hints

enum : int { CS_FREE = 0, CS_ACTIVE = 1, CS_PARKED = 2, CS_QUEUED = 3, CS_DONE = 4 };
enum : int { T_RESUME = 0, T_POP = 2 };

// Lane modes.  Each issues exactly one round of memory operations per sampler
// round, and all lanes' operations are in flight together.
enum : int {
    M_IDLE = 0,    // no work
    M_LOOK = 1,    // look at `tgt` and claim it if free (first publishing the head's
                   // new arrow if one was drawn)
    M_PARK = 2,    // join the waiter list of `tgt` if its tag word is still `seen`
    M_NEED = 3,    // set the need bit of start vertex `tgt` if its tag word is still `seen`
    M_ADJ = 4,     // the drawn neighbour lies beyond the inline ones: fetch it
    M_ERASE0 = 5,  // popping: load the kept vertex `tgt` (the new head)
    M_ERASE = 6,   // popping: free `tgt`, follow next until `stopv`
    M_FETCH = 7    // lean looks: load the arrow word and graph record of the head just claimed
};

template <int CH>
struct SamplerShared {
    int32_t block[CH];   // parked: vertex the head's arrow points at
    int16_t up[CH];      // parked: chain owning `block`
    int16_t wnext[CH];   // parked: next / previous chain parked on the same vertex (-1: none)
    int16_t wprev[CH];
    int8_t state[CH];    // CS_*
    int16_t fin[CH];     // last generation of the chain id whose path joined the tree (-1: none);
                         // the id's current generation is fin + 1
    int16_t ring[CH];    // free chain ids, taken first in, first out (so generations grow evenly)
    int32_t hint[HINTS];
};

struct SamplerWS {
    uint64_t *tagw;
    uint64_t *arrow;
    int32_t *rq;   // restart ring (n entries)
    int4 *queue;   // ready tasks (CH entries): {chain, kind, e, stop}
    int32_t *start; // chain start vertices (CH entries)
};

// Cooperative cycle popping of one sample by one wavefront.
//
// Every chain runs Wilson's loop-erased walk with loops popped explicitly
// (each vertex of a popped cycle becomes free and draws its next arrow when
// revisited).  Parked chains form a wait-for forest (chain -> owner of the
// vertex it points at); when a park closes a cycle in it, that is a cycle of
// current arrows spanning several chains, and it is popped as a whole.  Only
// genuine cycles of current arrows are ever popped, so the result is the
// cycle-popping outcome of the arrow stacks: independent of timing, of
// `walkers`, of the chain table and of which free vertices are started.
//
// A round: idle lanes take work; every busy lane issues its memory operations
// (one dependent round trip); the results are applied (draws from the head's
// inline neighbours, wakes, pushes); chains that reached the tree finish, with
// the parked chains that wait on them; newly parked chains are checked for a
// cycle of the wait-for forest, all in lockstep.
//
// Returns the total number of draws, or -1 (error recorded in ctl).
template <int CH, bool LEAN>
__device__ int64_t sample_tree(const GraphDev &g, const SamplerWS &ws, SamplerShared<CH> &sh,
                               uint64_t seed, uint64_t s, int walkers, int64_t iter_cap,
                               int32_t *ctl, int idx, int64_t *iters_used, int32_t root_u,
                               int32_t root_v) {
    const int lane = threadIdx.x;
    const int n = g.n, root = g.root;
    const bool two_roots = root_u >= 0;  // start from {u, v} instead of {root}
    uint64_t *__restrict__ tagw = ws.tagw;
    uint64_t *__restrict__ arw = ws.arrow;
    for (int v = lane; v < n; v += WAVE) {
        const bool in_tree = two_roots ? (v == root_u || v == root_v) : v == root;
        astore(&tagw[v], (uint64_t)(in_tree ? T_TREE : T_FREE));
        astore(&arw[v], arrow_of(-1, 0));
    }
    for (int c = lane; c < CH; c += WAVE) {
        sh.state[c] = CS_FREE;
        sh.fin[c] = -1;
        sh.ring[c] = (int16_t)c;
    }
    fence_wg();
    __syncthreads();

    const bool worker = lane < walkers;
    int mode = M_IDLE, chain = -1, cur = -1, tgt = -1, stopv = -1;
    uint32_t ctag = 0, dcur = 0;
    bool haspath = false;  // M_LOOK: the chain has a path (not a fresh start)
    bool pend = false;     // M_LOOK: publish arrow (cur -> tgt, dcur) first
    uint64_t seen = 0;     // M_PARK / M_NEED: expected tag word
    int adjpos = 0;        // M_ADJ: CSR position of the drawn neighbour
    // graph record of the head `cur`: CSR offset, degree, first neighbours (plain scalars,
    // so that the record stays in registers)
    int hoff = 0, hdeg = 0, hn0 = -1, hn1 = -1, hn2 = -1, hn3 = -1, hn4 = -1, hn5 = -1;
    // wave-uniform bookkeeping
    int next_start = 0, q_head = 0, q_tail = 0, f_head = 0, f_tail = CH, parked = 0, hint_top = 0;
    int64_t rq_head = 0, rq_tail = 0;
    int64_t iters = 0, mysteps = 0;
    int err = 0;

    // tag of chain c's path in its current generation
    auto tag_of = [&](int c) __attribute__((always_inline)) {
        return T_CHAIN0 + (uint32_t)c + (uint32_t)CH * (uint32_t)(sh.fin[c] + 1);
    };
    // a tree vertex: a start vertex, or on a path whose generation has joined the tree
    auto in_tree = [&](uint32_t t) __attribute__((always_inline)) {
        if (t < T_CHAIN0) return t == T_TREE;
        const uint32_t x = t - T_CHAIN0;
        return (int)(x / (uint32_t)CH) <= (int)sh.fin[x % (uint32_t)CH];
    };

    // the head `cur` (its graph record in registers, dcur draws so far) draws its next arrow;
    // called once per round for the lanes that set `drawing`
    auto draw = [&]() __attribute__((always_inline)) {
        const uint32_t deg = (uint32_t)hdeg;
        const uint32_t j = arrow_slot(seed, s, (uint32_t)cur, dcur, deg);
        mysteps++;
        dcur += 1;
        haspath = true;
        if (j < (uint32_t)VREC_INLINE) {
            // select in registers: pairs first, then the pair (an indexed read of the
            // record would place it in scratch memory)
            const bool odd = (j & 1u) != 0u;
            int p01 = odd ? hn1 : hn0;
            int p23 = odd ? hn3 : hn2;
            int p45 = odd ? hn5 : hn4;
            asm volatile("" : "+v"(p01), "+v"(p23), "+v"(p45));
            tgt = j < 2u ? p01 : (j < 4u ? p23 : p45);
            pend = true;
            mode = M_LOOK;
        } else {
            adjpos = hoff + (int)j;
            mode = M_ADJ;
        }
    };

    while (true) {
        // ---- phase 0: idle lanes take tasks, restarts, fresh starts, then hints
        {
            const uint64_t idle = __ballot(worker && mode == M_IDLE);
            const int nidle = __popcll(idle);
            const int take_q = min(nidle, q_tail - q_head);
            int left = nidle - take_q, room = f_tail - f_head;
            const int take_r = (int)min((int64_t)min(left, room), rq_tail - rq_head);
            left -= take_r; room -= take_r;
            const int take_s = min(min(left, room), n - next_start);
            left -= take_s; room -= take_s;
            const int take_h = min(min(left, room), hint_top);
            if (worker && mode == M_IDLE) {
                const int r = rank_in(idle);
                const int k = r - take_q;
                pend = false;
                // a lane that takes work reads all four sources at clamped, always
                // valid indices and keeps the one it needs, so its loads and those of
                // the other lanes are in flight together; lanes that take nothing
                // read nothing (a round with nothing to take has no load here)
                int4 t = make_int4(0, 0, 0, 0);
                int32_t t_rq = 0, t_ord = 0, t_hint = 0;
                if (r < take_q + take_r + take_s + take_h) {
                    t = ws.queue[(q_head + max(0, min(r, take_q - 1))) & (CH - 1)];
                    t_rq = aload(&ws.rq[(rq_head + max(0, min(k, take_r - 1))) % n]);
                    t_ord = aload(&g.order[max(0, min(next_start + k - take_r, n - 1))]);
                    t_hint = sh.hint[max(0, min(hint_top - 1 - (k - take_r - take_s), HINTS - 1))];
                }
                if (r < take_q) {
                    chain = t.x;
                    ctag = tag_of(chain);
                    if (t.y == T_RESUME) {
                        tgt = t.z;
                        haspath = true;
                        mode = M_LOOK;
                    } else {
                        tgt = t.z;
                        stopv = t.w;
                        mode = M_ERASE0;
                    }
                } else if (k < take_r + take_s + take_h) {
                    chain = sh.ring[(f_head + k) & (CH - 1)];
                    ctag = tag_of(chain);
                    tgt = k < take_r ? t_rq : (k < take_r + take_s ? t_ord : t_hint);
                    astore(&ws.start[chain], tgt);
                    haspath = false;
                    mode = M_LOOK;
                }
                if (mode != M_IDLE) sh.state[chain] = CS_ACTIVE;
            }
            q_head += take_q;
            rq_head += take_r;
            next_start += take_s;
            hint_top -= take_h;
            f_head += take_r + take_s + take_h;
        }
        if (__ballot(mode != M_IDLE) == 0ull) {
            if (next_start < n || q_tail != q_head || parked != 0 || rq_tail != rq_head)
                err = DEV_PROTOCOL;
            break;
        }
        if (++iters > iter_cap) err = DEV_LIMIT;
        if (err == 0 && mode != M_IDLE && mode != M_ADJ && (unsigned)tgt >= (unsigned)n)
            err = DEV_PROTOCOL;
        if (err == 0 && mode == M_ADJ && (unsigned)adjpos >= (unsigned)g.two_m) err = DEV_PROTOCOL;
        const int m0 = err == 0 ? mode : M_IDLE;

        // ---- memory: every lane issues its operations before any result is used
        const bool do_cas = m0 == M_LOOK || m0 == M_PARK || m0 == M_NEED;
        const bool do_xchg = m0 == M_ERASE;
        // a lean look at a walk's next vertex is the claim alone: most such looks
        // meet the tree, and a claimed vertex's arrow word and record are fetched
        // in the next round (M_FETCH)
        // (LEAN: a compile-time choice, so that a kernel without lean looks carries none of it)
        const bool thin = LEAN && m0 == M_LOOK && haspath;
        const bool fetch = LEAN && m0 == M_FETCH;
        const bool do_arrow = (m0 == M_LOOK && !thin) || m0 == M_ERASE0 || fetch || do_xchg;
        const bool do_rec = (m0 == M_LOOK && !thin) || m0 == M_ERASE0 || fetch;
        if (m0 == M_LOOK && pend) astore(&arw[cur], arrow_of(tgt, dcur));
        int4 r0 = make_int4(0, 0, 0, 0), r1 = make_int4(0, 0, 0, 0);
        const int rv = fetch ? cur : tgt;  // the vertex whose words are read
        if (do_rec) {
            r0 = g.vrec[2 * (size_t)rv];
            r1 = g.vrec[2 * (size_t)rv + 1];
        }
        // (each operation returns into a register of its own: a shared one would make
        // every later issue wait for the earlier operations' results)
        uint64_t o_cas = 0, o_xchg = 0, o_tag = 0;
        if (do_cas) {
            const uint64_t expect = m0 == M_LOOK ? (uint64_t)T_FREE : seen;
            const uint64_t want = m0 == M_LOOK ? (uint64_t)ctag
                                : m0 == M_PARK ? ((seen & 0xffffffffull) | ((uint64_t)(chain + 1) << 32))
                                               : (seen | TW_NEED);
            o_cas = acas(&tagw[tgt], expect, want);
        }
        if (do_xchg)
            o_xchg = __hip_atomic_exchange(&tagw[tgt], (uint64_t)T_FREE, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        if (m0 == M_ERASE0) o_tag = aload(&tagw[tgt]);
        uint64_t ar = 0;
        if (do_arrow) ar = aload(&arw[rv]);
        auto take_record = [&]() __attribute__((always_inline)) {
            hoff = r0.x; hdeg = r0.y; hn0 = r0.z; hn1 = r0.w;
            hn2 = r1.x; hn3 = r1.y; hn4 = r1.z; hn5 = r1.w;
        };
        int32_t y = -1;
        if (m0 == M_ADJ) y = g.adj[adjpos];
        const uint64_t o64 = do_cas ? o_cas : (do_xchg ? o_xchg : o_tag);

        // ---- apply the results
        bool retire = false, park = false, drawing = false, finish = false;
        int park_head = -1;
        int wake_kind = -1, wake_vtx = -1, wake_head = -1, restart_vtx = -1, hint_vtx = -1;
        const uint32_t old = (uint32_t)o64;
        const uint32_t tg = old & TW_TAG;
        const int32_t nt = (int32_t)(uint32_t)ar;
        const uint32_t dt = (uint32_t)(ar >> 32);
        if (m0 == M_LOOK) {
            const bool drew = pend;  // the arrow into tgt was just published
            pend = false;
            if (old == T_FREE) {
                // claimed: the new head draws at once (after a lean look, next round)
                cur = tgt;
                if (thin) {
                    mode = M_FETCH;
                } else {
                    dcur = dt;
                    take_record();
                    drawing = true;
                }
            } else if (tg == ctag) {
                // own path: the new arrow closed a loop at tgt; pop it, keep tgt as head
                if (!drew) err = DEV_PROTOCOL;
                stopv = tgt;
                if (thin) {
                    mode = M_ERASE0;  // reads tgt's words, then erases from its arrow on
                } else {
                    cur = tgt;
                    dcur = dt;
                    take_record();
                    tgt = nt;
                    mode = M_ERASE;
                }
            } else if (in_tree(tg)) {
                if (haspath) finish = true;  // the path reaches the tree and joins it
                else retire = true;          // a fresh chain whose start is already in the tree
            } else if (tg >= T_CHAIN0) {
                seen = o64;
                mode = haspath ? M_PARK : M_NEED;
            } else {
                err = DEV_PROTOCOL;
            }
        } else if (m0 == M_PARK || m0 == M_NEED) {
            if (o64 == seen) {
                if (m0 == M_PARK) {
                    park = true;  // joined the list; recorded below
                    park_head = (int)(seen >> 32) - 1;
                } else {
                    retire = true;  // need mark set: the fresh chain has nothing to retrace
                }
            } else if (o64 == (uint64_t)T_FREE) {
                mode = M_LOOK;  // popped meanwhile: look again
            } else if (in_tree(tg)) {
                if (m0 == M_PARK) finish = true;
                else retire = true;
            } else if (tg >= T_CHAIN0 && tg != ctag) {
                seen = o64;  // another park or a new owner: try again
            } else {
                err = DEV_PROTOCOL;
            }
        } else if (m0 == M_ADJ) {
            tgt = y;
            pend = true;
            mode = M_LOOK;
        } else if (m0 == M_ERASE) {
            if (tg != ctag) err = DEV_PROTOCOL;
            wake_head = (int)(o64 >> 32) - 1;
            if (wake_head >= 0) { wake_kind = T_RESUME; wake_vtx = tgt; }
            if (old & TW_NEED) restart_vtx = tgt;
            else hint_vtx = tgt;
            if (nt == stopv) drawing = true; else tgt = nt;
        } else if (m0 == M_ERASE0) {
            if (tg != ctag) err = DEV_PROTOCOL;
            cur = tgt;
            dcur = dt;
            take_record();
            if (nt == stopv) drawing = true;
            else { mode = M_ERASE; tgt = nt; }
        } else if (fetch) {
            dcur = dt;
            take_record();
            drawing = true;
        }
        if (drawing) draw();
        // paths that reached the tree join it: their generation is finished
        auto finish_chain = [&](int c) __attribute__((always_inline)) {
            if ((int)sh.fin[c] + 1 > GEN_MAX) err = DEV_LIMIT;
            sh.fin[c] = (int16_t)(sh.fin[c] + 1);
            sh.state[c] = CS_DONE;
        };
        if (finish) finish_chain(chain);
        __syncthreads();
        // a new park on a path that has joined the tree (in this round, or since its
        // owner was looked at) joins the tree with it instead
        if (park && in_tree(tg)) {
            park = false;
            finish = true;
            finish_chain(chain);
        }
        // new parks join their vertex's list before any wake walks a list
        if (park) {
            int h = park_head;
            if ((unsigned)(h + 1) > (unsigned)CH) { err = DEV_PROTOCOL; h = -1; }
            sh.wnext[chain] = (int16_t)h;
            sh.wprev[chain] = -1;
            if (h >= 0) sh.wprev[h] = (int16_t)chain;
            sh.block[chain] = tgt;
            sh.up[chain] = (int16_t)((tg - T_CHAIN0) % (uint32_t)CH);
            sh.state[chain] = CS_PARKED;
        }
        // popped vertices: need-restarts to the restart ring, the rest offered as hints
        {
            const uint64_t qm = __ballot(restart_vtx >= 0);
            if (restart_vtx >= 0) astore(&ws.rq[(rq_tail + rank_in(qm)) % n], (int32_t)restart_vtx);
            rq_tail += __popcll(qm);
            const uint64_t hm = __ballot(hint_vtx >= 0);
            if (hint_vtx >= 0) {
                const int k = hint_top + rank_in(hm);
                if (k < HINTS) sh.hint[k] = hint_vtx;
            }
            hint_top = min(HINTS, hint_top + __popcll(hm));
        }
        // retired chains return to the free ring
        {
            const uint64_t rm = __ballot(retire);
            if (retire) {
                sh.ring[(f_tail + rank_in(rm)) & (CH - 1)] = (int16_t)chain;
                sh.state[chain] = CS_FREE;
                mode = M_IDLE;
                chain = -1;
            }
            f_tail += __popcll(rm);
        }
        const uint64_t pm0 = __ballot(park);
        parked += __popcll(pm0);
        __syncthreads();
        // the chains whose walk reached the tree go back to the free ring at once; a
        // parked chain whose head's arrow points into a path that joined the tree
        // joins it too, transitively (a scan of the chain table per step, only
        // while chains are parked), and goes back to the ring as it is found.
        // Their state reads "done" until the closure is over.
        const uint64_t fm = __ballot(finish);
        if (fm != 0ull) {
            const int f0 = f_tail;
            if (finish) sh.ring[(f_tail + rank_in(fm)) & (CH - 1)] = (int16_t)chain;
            f_tail += __popcll(fm);
            __syncthreads();
            for (int pass = 0; parked > 0; ++pass) {
                int tot = 0;
                for (int c0 = 0; c0 < CH; c0 += WAVE) {
                    const int c = c0 + lane;
                    const bool join = sh.state[c] == CS_PARKED && sh.state[sh.up[c]] == CS_DONE;
                    const uint64_t jm = __ballot(join);
                    if (join) {
                        finish_chain(c);
                        sh.ring[(f_tail + rank_in(jm)) & (CH - 1)] = (int16_t)c;
                    }
                    f_tail += __popcll(jm);
                    tot += __popcll(jm);
                }
                __syncthreads();
                parked -= tot;
                if (tot == 0) break;
                if (pass > CH) { err = DEV_PROTOCOL; break; }
            }
            for (int i = f0 + lane; i < f_tail; i += WAVE) sh.state[sh.ring[i & (CH - 1)]] = CS_FREE;
            if (finish) {
                mode = M_IDLE;
                chain = -1;
            }
            __syncthreads();
        }
        // wake the chains parked on vertices that were popped or joined the tree:
        // each such lane walks the list its atomic detached, one chain per pass
        if ((unsigned)(wake_head + 1) > (unsigned)CH) { err = DEV_PROTOCOL; wake_head = -1; }
#pragma unroll 1
        for (int pass = 0;; ++pass) {
            const uint64_t wm = __ballot(wake_head >= 0);
            if (wm == 0ull) break;
            if (pass == CH) {  // longer than the chain table: the lists are broken
                err = DEV_PROTOCOL;
                break;
            }
            if (wake_head >= 0) {
                const int c = wake_head;
                if (sh.state[c] != CS_PARKED || sh.block[c] != wake_vtx) err = DEV_PROTOCOL;
                ws.queue[(q_tail + rank_in(wm)) & (CH - 1)] = make_int4(c, wake_kind, wake_vtx, 0);
                sh.state[c] = CS_QUEUED;
                wake_head = sh.wnext[c];
                if ((unsigned)(wake_head + 1) > (unsigned)CH) { err = DEV_PROTOCOL; wake_head = -1; }
            }
            q_tail += __popcll(wm);
            parked -= __popcll(wm);
        }
        __syncthreads();

        // ---- new parks: each looks for a cycle of parked chains through its own
        // new owner link, all lanes in lockstep (a chain woken above is no longer
        // parked).  A walk that runs into a cycle closed by another new park
        // stops there (Brent's cycle finding), so every walk ends within a few
        // times the number of chains.  A cycle is found by each new park on it;
        // its smallest chain index identifies it, and the lowest such lane pops
        // it, one cycle at a time.  (Most rounds park nothing and skip this.)
        if (pm0 != 0ull) {
            const int c = chain;
            bool walking = ((pm0 >> lane) & 1ull) != 0ull && sh.state[c] == CS_PARKED;
            bool on_cycle = false;
            int hare = 0, tort = 0, cmin = c, power = 1, lam = 1;
            if (walking) {
                const int x0 = sh.up[c];
                if (sh.state[x0] != CS_PARKED) {
                    walking = false;
                } else {
                    cmin = min(c, x0);
                    tort = x0;
                    hare = sh.up[x0];
                }
            }
#pragma unroll 1
            for (int step = 0; __ballot(walking) != 0ull; ++step) {
                if (walking) {
                    if (hare == c) {
                        on_cycle = true;
                        walking = false;
                    } else if (sh.state[hare] != CS_PARKED || hare == tort) {
                        walking = false;  // reaches a walking chain, or another new cycle
                    } else if (step >= 4 * CH) {
                        err = DEV_PROTOCOL;  // longer than any walk through the chain table
                        walking = false;
                    } else {
                        cmin = min(cmin, hare);
                        if (power == lam) {
                            tort = hare;
                            power <<= 1;
                            lam = 0;
                        }
                        hare = sh.up[hare];
                        ++lam;
                    }
                }
            }
            uint64_t todo = __ballot(on_cycle);
            while (todo != 0ull) {
                const int L = __ffsll((unsigned long long)todo) - 1;
                const int key = __shfl(cmin, L);
                todo &= ~__ballot(on_cycle && cmin == key);
                int ncyc = 0;
                if (lane == L) {
                    // the chains c -> up(c) -> ... -> c form a cycle of arrows: pop all
                    // of them; each keeps the vertex where its predecessor entered it
                    // and leaves the waiter list of the vertex it was parked on
                    int prev = c, m;
                    do {
                        m = sh.up[prev];
                        const int wp = sh.wprev[m], wn = sh.wnext[m];
                        if (wp >= 0) sh.wnext[wp] = (int16_t)wn;
                        else astore(tag_high(&tagw[sh.block[m]]), (uint32_t)(wn + 1));
                        if (wn >= 0) sh.wprev[wn] = (int16_t)wp;
                        ws.queue[(q_tail + ncyc) & (CH - 1)] = make_int4(m, T_POP, sh.block[prev], sh.block[m]);
                        sh.state[m] = CS_QUEUED;
                        ++ncyc;
                        prev = m;
                    } while (m != c && ncyc <= CH);
                }
                ncyc = __shfl(ncyc, L);
                parked -= ncyc;
                q_tail += ncyc;
                __syncthreads();
            }
            if (((pm0 >> lane) & 1ull) != 0ull) {
                mode = M_IDLE;
                chain = -1;
            }
        }
        fence_wg();
        if (__ballot(err != 0) != 0ull) break;
    }
    const int e = wave_max(err);
    if (e != 0) {
        report_error(ctl, e, idx);
        return -1;
    }
    *iters_used = iters;
    return wave_sum(mysteps);
}

// --------------------------------------------------------- tree traversal

// The numbered tree: one 16-byte record per vertex, two 8-byte words, so that
// every step of the numbering touches one line per vertex it visits:
//   rec[2v]     pending children << 44 | volume while the volumes are summed
//               (starting at deg(v)); tin(v) + vol(v) once the numbering is done
//   rec[2v + 1] parent (low half, -1 at the root) | deg(v) (high half) until the
//               top-down step, then parent | tin(v)
struct SlotPtrs {
    SamplerWS ws;
    uint64_t *rec;
    int4 *ord;             // finished vertices {v, parent, vol, offset in the parent's interval} in
                           // completion order; the leaves {v, parent, deg, 0} wait at its end
    int32_t *grp;
    int64_t *fen;
};

__device__ __forceinline__ int32_t rec_parent(const uint64_t *rec, int v) {
    return (int32_t)(uint32_t)aload(&rec[2 * (size_t)v + 1]);
}
// The numbering of a vertex once it is complete: tin, vol and tree parent.
struct TNum {
    uint32_t tin, vol;
    int32_t par;
};
__device__ __forceinline__ TNum rec_num(const uint64_t *rec, int v) {
    const uint64_t w = aload(&rec[2 * (size_t)v]), h = aload(&rec[2 * (size_t)v + 1]);
    TNum t;
    t.tin = (uint32_t)(h >> 32);
    t.vol = (uint32_t)(w - (h >> 32));
    t.par = (int32_t)(uint32_t)h;
    return t;
}
__device__ __forceinline__ uint32_t rec_tin(const uint64_t *rec, int v) {
    return (uint32_t)(aload(&rec[2 * (size_t)v + 1]) >> 32);
}

// Vertices each lane keeps in flight in the tree numbering: the memory
// operations of one step are issued together, so a wavefront has this many
// times as many requests outstanding as it has lanes.  The streaming passes
// take twice as many.
constexpr int NB = 4;
constexpr int NBS = 8;

constexpr uint64_t PEND_ONE = 1ull << 44;
constexpr uint64_t VOL_MASK = PEND_ONE - 1;

__device__ __forceinline__ uint32_t degree(const GraphDev &g, int v) {
    return (uint32_t)(g.off[v + 1] - g.off[v]);
}

// Fenwick tree over positions 0..2m storing a difference array.
__device__ __forceinline__ void fen_point_add(int64_t *fen, int64_t len, int64_t pos, int64_t val) {
    if (pos < 0) pos = 0;
    for (int64_t i = pos + 1; i < len; i += i & (-i)) afetch_add(&fen[i], val);
}
__device__ __forceinline__ void fen_range_add(int64_t *fen, int64_t len, int64_t lo, int64_t hi,
                                              int64_t val) {
    if (val == 0 || hi <= lo) return;
    fen_point_add(fen, len, lo, val);
    fen_point_add(fen, len, hi, -val);
}
__device__ __forceinline__ int64_t fen_prefix(const int64_t *fen, int64_t len, int64_t pos) {
    int64_t i = pos + 1;
    if (i >= len) i = len - 1;
    int64_t sum = 0;
    for (; i > 0; i -= i & (-i)) sum += aload(&fen[i]);
    return sum;
}

// The two contributions attached to tau0 vertex x (Theorem 3.4), as
// ranges of tin with a weight, active for every u in Sub(tau0, x):
//   forward : p(x) = p0(x)          -> +(2m - vol(x)) on Sub(tau, x)
//   reverse : p(p0(x)) = x, p0(x)!=r -> -(2m - vol(p0(x))) on Sub(tau, p0(x))
struct Items {
    uint32_t flo, fhi, rlo, rhi;
    int64_t fw, rw;
};
__device__ __forceinline__ Items items_of(const GraphDev &g, const uint64_t *rec, int x) {
    Items it{0u, 0u, 0u, 0u, 0, 0};
    if (x == g.root) return it;
    const TNum nx = rec_num(rec, x);
    const int z = g.p0[x];
    if (nx.par == z) {
        it.flo = nx.tin; it.fhi = nx.tin + nx.vol; it.fw = g.two_m - (int64_t)nx.vol;
    }
    if (z != g.root) {
        const TNum nz = rec_num(rec, z);
        if (nz.par == x) {
            it.rlo = nz.tin; it.rhi = nz.tin + nz.vol; it.rw = (int64_t)nz.vol - g.two_m;
        }
    }
    return it;
}
__device__ __forceinline__ int64_t items_at(const Items &it, uint32_t t) {
    int64_t s = 0;
    if (it.flo <= t && t < it.fhi) s += it.fw;
    if (it.rlo <= t && t < it.rhi) s += it.rw;
    return s;
}

// Volumes and the volume-weighted preorder of the tree whose parents are in
// rec (rec[2v] = deg(v), rec[2v+1] = parent | deg(v) << 32 already).  Returns
// false if the parents do not form a tree rooted at r.
//
// Bottom-up: each lane carries up to NB finished vertices; a carrier pushes
// its vertex's volume into the parent's word with one atomic, and the last
// child to arrive carries the parent on in the next round.  The volume part
// the atomic returns is the parent's degree plus the volumes of the siblings
// that arrived before: the vertex's offset in its parent's interval.  Every
// round's finished vertices form a completion group.  Top-down: the groups in
// reverse order (a parent always finishes in a later group than its
// children); a vertex's tin is its parent's tin plus its offset.
__device__ bool tree_numbering(const GraphDev &g, const SlotPtrs &sp) {
    const int lane = threadIdx.x;
    const int n = g.n;
    // one PEND_ONE per child in the parent's word
    for (int b = 0; b < n; b += WAVE * NBS) {
        int32_t p[NBS];
#pragma unroll
        for (int k = 0; k < NBS; ++k) {
            const int v = b + k * WAVE + lane;
            p[k] = v < n ? rec_parent(sp.rec, v) : -1;
        }
#pragma unroll
        for (int k = 0; k < NBS; ++k)
            if (p[k] >= 0) afetch_add(&sp.rec[2 * (size_t)p[k]], PEND_ONE);
    }
    fence_wg();
    // leaves {v, parent, deg, 0}: leaf number j at ord[n - 1 - j]
    int L = 0;
    for (int b = 0; b < n; b += WAVE * NBS) {
        uint64_t w[NBS], h[NBS];
#pragma unroll
        for (int k = 0; k < NBS; ++k) {
            const int v = b + k * WAVE + lane;
            w[k] = v < n ? aload(&sp.rec[2 * (size_t)v]) : PEND_ONE;  // past the end: not a leaf
            h[k] = v < n ? aload(&sp.rec[2 * (size_t)v + 1]) : 0;
        }
#pragma unroll
        for (int k = 0; k < NBS; ++k) {
            const bool leaf = (w[k] >> 44) == 0;
            const uint64_t m = __ballot(leaf);
            if (leaf)
                sp.ord[n - 1 - (L + rank_in(m))] = make_int4(b + k * WAVE + lane, (int32_t)(uint32_t)h[k],
                                                             (int)(w[k] & VOL_MASK), 0);
            L += __popcll(m);
        }
    }
    fence_wg();
    // bottom-up.  Leaves are taken from the low end of their block, ord[n-L ..]:
    // the finished entries written at ord[0 .. nord) never reach an untaken leaf,
    // since nord + (leaves not yet taken) <= n.
    int cv[NB], cp[NB];
    uint64_t cval[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) { cv[k] = -1; cp[k] = -1; cval[k] = 0; }
    int li = 0, nord = 0, ngrp = 0;
    while (true) {
        if (li < L) {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint64_t freem = __ballot(cv[k] < 0);
                const int j = li + rank_in(freem);
                if (cv[k] < 0 && j < L) {
                    const int4 e = sp.ord[n - L + j];
                    cv[k] = e.x;
                    cp[k] = e.y;
                    cval[k] = (uint64_t)(uint32_t)e.z;
                }
                li = min(L, li + (int)__popcll(freem));
            }
        }
        uint64_t busy = 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) busy |= __ballot(cv[k] >= 0);
        if (busy == 0ull) break;
        if (lane == 0) astore(&sp.grp[ngrp], nord);
        ngrp++;
        uint64_t old[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            old[k] = 0;
            if (cv[k] >= 0 && cp[k] >= 0) old[k] = afetch_add(&sp.rec[2 * (size_t)cp[k]], cval[k] - PEND_ONE);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const uint64_t bm = __ballot(cv[k] >= 0);
            if (cv[k] >= 0)
                sp.ord[nord + rank_in(bm)] = make_int4(cv[k], cp[k], (int)cval[k], (int)(uint32_t)(old[k] & VOL_MASK));
            nord += __popcll(bm);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const bool last = cv[k] >= 0 && cp[k] >= 0 && (old[k] >> 44) == 1;
            cv[k] = last ? cp[k] : -1;
            if (last) cval[k] = (old[k] & VOL_MASK) + cval[k];
        }
        // the new carrier's parent, from the record line the atomic just used
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (cv[k] >= 0) cp[k] = rec_parent(sp.rec, cv[k]);
        if (nord > n) break;  // more entries than vertices: not a tree
    }
    if (lane == 0) astore(&sp.grp[ngrp], nord);
    fence_wg();
    if (nord != n) return false;
    // top-down; the group boundaries are read 64 at a time
    for (int g0 = ngrp - 1; g0 >= 0; g0 -= WAVE) {
        const int bnd = g0 - lane >= 0 ? aload(&sp.grp[g0 - lane]) : 0;
        const int nb = min(WAVE, g0 + 1);
        int hi = aload(&sp.grp[g0 + 1]);
        for (int t = 0; t < nb; ++t) {
            const int lo = __shfl(bnd, t);
            for (int i0 = lo; i0 < hi; i0 += WAVE * NB) {
                int4 e[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const int i = i0 + k * WAVE + lane;
                    e[k] = i < hi ? sp.ord[i] : make_int4(-1, -1, 0, 0);
                }
                // tin = the parent's tin (written by its own group) + the offset the
                // bottom-up atomic returned
                uint64_t tin[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    tin[k] = 0;
                    if (e[k].x >= 0 && e[k].y >= 0) tin[k] = (uint64_t)rec_tin(sp.rec, e[k].y) + (uint32_t)e[k].w;
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    if (e[k].x < 0) continue;
                    astore(&sp.rec[2 * (size_t)e[k].x], tin[k] + (uint64_t)(uint32_t)e[k].z);
                    astore(&sp.rec[2 * (size_t)e[k].x + 1], (uint64_t)(uint32_t)e[k].y | (tin[k] << 32));
                }
            }
            fence_wg();  // the next group reads the intervals of this one
            hi = lo;
        }
    }
    return true;
}

// f by walking each vertex's tau0 ancestors (Theorem 3.4 as a sum over
// vertices u of d(u) q(u): every tau0 edge x -> p0(x) on u's tau0 path adds
// 2m - vol(x) when tau uses it in the same direction and x is a tau ancestor
// of u, and subtracts 2m - vol(p0(x)) when tau uses it the other way and
// p0(x) (not the root) is a tau ancestor of u).
//
// With the graph's ancestor table (shallow tau0: anc0[i n + u] is the
// (i+1)-th tau0 ancestor of u, -1 past the root) every record a vertex needs
// is loaded at once; otherwise the walk follows p0 step by step.

template <int D>
__device__ __forceinline__ int64_t q_of_table(const GraphDev &g, const SlotPtrs &sp, int u) {
    const int root = g.root;
    const int64_t two_m = g.two_m;
    const size_t n = (size_t)g.n;
    int z[D];
#pragma unroll
    for (int i = 0; i < D; ++i) z[i] = g.anc0[(size_t)i * n + (size_t)u];
    TNum nz[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        nz[i] = TNum{0u, 0u, -2};
        if (z[i] >= 0 && z[i] != root) nz[i] = rec_num(sp.rec, z[i]);
    }
    const TNum nu = rec_num(sp.rec, u);
    const uint32_t tu = nu.tin;
    int x = u;
    TNum nx = nu;
    int64_t q = 0;
    bool go = u != root;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (go && z[i] >= 0) {
            if (nx.par == z[i]) {
                if (nx.tin <= tu && tu < nx.tin + nx.vol) q += two_m - (int64_t)nx.vol;
            }
            if (z[i] == root) {
                go = false;
            } else {
                if (nz[i].par == x) {
                    if (nz[i].tin <= tu && tu < nz[i].tin + nz[i].vol) q -= two_m - (int64_t)nz[i].vol;
                }
                x = z[i];
                nx = nz[i];
            }
        }
    }
    return q;
}

// U vertices per lane and step (their loads in flight together); the deeper
// table takes one, to keep the kernel's register count at its occupancy (a
// table of more than 8 levels would not fit it, so deeper trees follow p0).
template <int D, int U>
__device__ int64_t f_walk_table(const GraphDev &g, const SlotPtrs &sp) {
    const int lane = threadIdx.x;
    const int n = g.n;
    int64_t acc = 0;
    for (int b = 0; b < n; b += U * WAVE) {
        int64_t q[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int u = b + k * WAVE + lane;
            q[k] = u < n ? q_of_table<D>(g, sp, u) : 0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int u = b + k * WAVE + lane;
            if (u < n) acc += (int64_t)degree(g, u) * q[k];
        }
    }
    return wave_sum(acc);
}

__device__ int64_t f_walk(const GraphDev &g, const SlotPtrs &sp) {
    if (g.anc0 && g.anc_depth <= 4) return f_walk_table<4, 2>(g, sp);
    if (g.anc0 && g.anc_depth <= 8) return f_walk_table<8, 1>(g, sp);
    const int lane = threadIdx.x;
    const int n = g.n, root = g.root;
    const int64_t two_m = g.two_m;
    int64_t acc = 0;
    for (int u = lane; u < n; u += WAVE) {
        const TNum nu = rec_num(sp.rec, u);
        const uint32_t tu = nu.tin;
        int64_t q = 0;
        int x = u;
        TNum nx = nu;
        while (x != root) {
            const int z = g.p0[x];
            if (nx.par == z) {
                if (nx.tin <= tu && tu < nx.tin + nx.vol) q += two_m - (int64_t)nx.vol;
            }
            if (z == root) break;
            const TNum nz = rec_num(sp.rec, z);
            if (nz.par == x) {
                if (nz.tin <= tu && tu < nz.tin + nz.vol) q -= two_m - (int64_t)nz.vol;
            }
            x = z;
            nx = nz;
        }
        acc += (int64_t)degree(g, u) * q;
    }
    return wave_sum(acc);
}

// f by a tau0-preorder sweep, 64 preorder positions per step.  The Fenwick
// tree holds the items of every tau0 vertex whose subtree started before the
// step and is still open; items of the step's own vertices and of subtrees
// closing inside the step are handled exactly from LDS.  The tree returns
// to all zeros at the end of the sweep.
struct SweepShared {
    Items it[WAVE];
    int32_t out[WAVE];
    Items eit[WAVE];
    int32_t eout[WAVE];
};

__device__ int64_t f_sweep(const GraphDev &g, const SlotPtrs &sp, int64_t fen_len, SweepShared &ss) {
    Items *sh_it = ss.it;
    int32_t *sh_out = ss.out;
    Items *se_it = ss.eit;
    int32_t *se_out = ss.eout;
    const int lane = threadIdx.x;
    const int n = g.n;
    int64_t acc = 0;
    int blk = 0;
    for (int P0 = 0; P0 < n; P0 += WAVE, ++blk) {
        const int p = P0 + lane;
        const bool valid = p < n;
        Items it{0u, 0u, 0u, 0u, 0, 0};
        int32_t o = -1;
        uint32_t tu = 0;
        int u = g.root;
        if (valid) {
            u = g.pre0[p];
            it = items_of(g, sp.rec, u);
            o = g.out0[u];
            tu = rec_tin(sp.rec, u);
        }
        int64_t S = valid ? fen_prefix(sp.fen, fen_len, tu) : 0;
        sh_it[lane] = it;
        sh_out[lane] = o;
        __syncthreads();
        if (valid) {
            for (int j = 0; j <= lane; ++j)
                if (sh_out[j] >= p) S += items_at(sh_it[j], tu);
        }
        const int e0 = g.eoff[blk], e1 = g.eoff[blk + 1];
        for (int c = e0; c < e1; c += WAVE) {
            const int k = c + lane;
            Items ex{0u, 0u, 0u, 0u, 0, 0};
            int32_t xo = -1;
            if (k < e1) {
                const int x = g.elist[k];
                ex = items_of(g, sp.rec, x);
                xo = g.out0[x];
            }
            se_it[lane] = ex;
            se_out[lane] = xo;
            __syncthreads();
            if (valid) {
                const int cnt = min(WAVE, e1 - c);
                for (int j = 0; j < cnt; ++j)
                    if (se_out[j] < p) S -= items_at(se_it[j], tu);
            }
            if (k < e1) {
                fen_range_add(sp.fen, fen_len, ex.flo, ex.fhi, -ex.fw);
                fen_range_add(sp.fen, fen_len, ex.rlo, ex.rhi, -ex.rw);
            }
            __syncthreads();
        }
        if (valid) {
            acc += (int64_t)degree(g, u) * S;
            if (o >= P0 + WAVE) {
                fen_range_add(sp.fen, fen_len, it.flo, it.fhi, it.fw);
                fen_range_add(sp.fen, fen_len, it.rlo, it.rhi, it.rw);
            }
        }
        fence_wg();
        __syncthreads();
    }
    return wave_sum(acc);
}

// Signed count of the edges of a fixed u -> v path that the tree's own u -> v
// path uses (+1 along the path's direction, -1 against it); its mean over
// uniform spanning trees is the effective resistance R(u, v) (Kirchhoff: the
// tree path's direction on an edge has mean equal to the unit current there,
// and currents summed along any u -> v path give the potential difference).
// Ancestry from the tree numbering: x is an ancestor of y (or y itself) iff
// tin(x) <= tin(y) < tin(x) + vol(x).
__device__ int64_t path_current(const SlotPtrs &sp, const int32_t *path, int len) {
    const int lane = threadIdx.x;
    const int u = path[0], v = path[len - 1];
    const uint32_t tu = rec_tin(sp.rec, u), tv = rec_tin(sp.rec, v);
    auto anc_u = [&](uint32_t t, uint32_t vol) { return t <= tu && tu < t + vol; };
    auto anc_v = [&](uint32_t t, uint32_t vol) { return t <= tv && tv < t + vol; };
    int64_t c = 0;
    for (int i = lane; i + 1 < len; i += WAVE) {
        const int a = path[i], b = path[i + 1];
        const TNum na = rec_num(sp.rec, a), nb = rec_num(sp.rec, b);
        const uint32_t ta = na.tin, va = na.vol, tb = nb.tin, vb = nb.vol;
        const int32_t pa = na.par, pb = nb.par;
        const bool up_a = anc_u(ta, va) && !anc_v(ta, va), up_b = anc_u(tb, vb) && !anc_v(tb, vb);
        const bool dn_a = anc_v(ta, va) && !anc_u(ta, va), dn_b = anc_v(tb, vb) && !anc_u(tb, vb);
        if ((up_a && pa == b) || (dn_b && pb == a)) c += 1;
        else if ((up_b && pb == a) || (dn_a && pa == b)) c -= 1;
    }
    return wave_sum(c);
}

// Number of graph edges {x, y} that join the two trees left when the tree
// edge {cut_u, cut_v} is removed (the side away from the root is Sub(tau, c)
// with c the child endpoint; membership from the tree numbering).  With
// relink, also cut-link (section 4.2): edge number j of them, in the order
// (x ascending, row order, x < y), with j drawn by Philox on counter
// (slot, serial, ISM_CTR_LO, ISM_CTR_HI), joins the two parts; the path from
// its inner endpoint up to c is reversed so the tree stays rooted at r.
__device__ int64_t crossing_edges(const GraphDev &g, const SlotPtrs &sp, const RunParams &rp, int32_t slot,
                                  int idx) {
    const int lane = threadIdx.x;
    const int n = g.n;
    const int a = rp.cut_u, b = rp.cut_v;
    const int32_t pa = rec_parent(sp.rec, a);
    const int32_t pb = rec_parent(sp.rec, b);
    const int c = pa == b ? a : (pb == a ? b : -1);
    if (c < 0) {
        report_error(rp.ctl, DEV_BADTREE, idx);
        return 0;
    }
    const TNum nc = rec_num(sp.rec, c);
    const uint32_t lo = nc.tin, hi = nc.tin + nc.vol;
    auto inside = [&](int x) {
        const uint32_t t = rec_tin(sp.rec, x);
        return lo <= t && t < hi;
    };
    auto row_count = [&](int x, bool ix) {
        int64_t k = 0;
        for (int64_t e = g.off[x]; e < g.off[x + 1]; ++e) {
            const int y = g.adj[e];
            if (y > x && inside(y) != ix) ++k;
        }
        return k;
    };
    int64_t cnt = 0;
    for (int x = lane; x < n; x += WAVE) cnt += row_count(x, inside(x));
    const int64_t total = wave_sum(cnt);
    if (!rp.relink) return total;
    if (total <= 0) {
        report_error(rp.ctl, DEV_BADTREE, idx);
        return 0;
    }
    const int64_t j = arrow_slot(rp.seed, ((uint64_t)ISM_CTR_HI << 32) | ISM_CTR_LO, rp.serial, (uint32_t)slot,
                                 (uint32_t)total);
    int64_t base = 0;
    for (int x0 = 0; x0 < n; x0 += WAVE) {
        const int x = x0 + lane;
        const bool ix = x < n && inside(x);
        const int64_t k = x < n ? row_count(x, ix) : 0;
        int64_t incl = k;
        for (int d = 1; d < WAVE; d <<= 1) {
            const int64_t t = __shfl_up(incl, d);
            if (lane >= d) incl += t;
        }
        const int64_t chunk = __shfl(incl, WAVE - 1);
        if (base + chunk > j) {
            if (k > 0 && base + incl - k <= j && j < base + incl) {
                int64_t r = j - (base + incl - k);
                int y = -1;
                for (int64_t e = g.off[x]; e < g.off[x + 1]; ++e) {
                    const int z = g.adj[e];
                    if (z > x && inside(z) != ix) {
                        if (r == 0) { y = z; break; }
                        --r;
                    }
                }
                if (y < 0) {
                    report_error(rp.ctl, DEV_BADTREE, idx);
                } else {
                    const int xi = ix ? x : y, yo = ix ? y : x;
                    int32_t *out = rp.parents_mut + (size_t)slot * (size_t)n;
                    int32_t prev = yo, z = xi;
                    for (int guard = 0; guard <= n; ++guard) {
                        const int32_t nz = rec_parent(sp.rec, z);
                        out[z] = prev;
                        if (z == c) break;
                        if (nz < 0 || nz >= n) {  // c is an ancestor of xi: not reached
                            report_error(rp.ctl, DEV_BADTREE, idx);
                            break;
                        }
                        prev = z;
                        z = nz;
                    }
                }
            }
            break;
        }
        base += chunk;
    }
    return total;
}

// ------------------------------------------------------------ the kernels

// The sampler and the sweep run one after the other: one LDS block serves both.
template <int CH>
union KernelShared {
    SamplerShared<CH> samp;
    SweepShared sweep;
};

// The per-slot arrays of workgroup blockIdx.x, each `stride` vertices long.
__device__ __forceinline__ SlotPtrs slot_ptrs(const SlotDev &sd, size_t stride) {
    SlotPtrs sp;
    const size_t b = (size_t)blockIdx.x;
    unsigned char *st = sd.state + b * (size_t)state_bytes((int64_t)stride);
    sp.ws.tagw = reinterpret_cast<uint64_t *>(st);
    sp.ws.arrow = reinterpret_cast<uint64_t *>(st + 8 * stride);
    sp.ws.rq = reinterpret_cast<int32_t *>(st + 16 * stride);
    sp.ws.queue = sd.queue + b * (size_t)sd.chains;
    sp.ws.start = sd.cstart + b * (size_t)sd.chains;
    sp.rec = sd.rec ? reinterpret_cast<uint64_t *>(sd.rec) + 2 * b * stride : nullptr;
    // the numbering's arrays reuse the sampler's block (dead once the parents are in rec)
    sp.ord = sd.rec ? reinterpret_cast<int4 *>(st) : nullptr;
    sp.grp = sd.rec ? reinterpret_cast<int32_t *>(st + 16 * stride) : nullptr;
    sp.fen = sd.fen ? sd.fen + b * (size_t)sd.fen_len : nullptr;
    return sp;
}

// One sample s (work item idx) of graph g through the whole path in the
// calling workgroup: the tree, then (except in RUN_SAMPLE) its numbering and
// f.  Returns false when the workgroup must stop (an error was recorded).
// CROSS: the instantiation for RUN_CROSS only (no sampler, no f), kept apart
// so that its code does not weigh on the sampler's register allocation.
template <int CH, bool CROSS, bool LEAN>
__device__ bool process_one(const GraphDev &g, const SlotPtrs &sp, KernelShared<CH> &lds, const RunParams &rp,
                            int64_t fen_len, int idx, uint64_t s) {
    const int lane = threadIdx.x;
    const size_t n = (size_t)g.n;
    int64_t steps = 0, iters = 0;
    if (!CROSS && (rp.mode == RUN_SAMPLE || rp.mode == RUN_ESTIMATE)) {
        steps = sample_tree<CH, LEAN>(g, sp.ws, lds.samp, rp.seed, s, rp.walkers, rp.iter_cap, rp.ctl, idx, &iters,
                                rp.root_u, rp.root_v);
        if (steps < 0) return false;
    }
    if (!CROSS && rp.mode == RUN_SAMPLE) {
        int32_t *po = rp.parents_out + (size_t)idx * n;
        uint32_t *co = rp.cnt_out ? rp.cnt_out + (size_t)idx * n : nullptr;
        for (int v = lane; v < g.n; v += WAVE) {
            const uint64_t ar = aload(&sp.ws.arrow[v]);
            po[v] = (int32_t)(uint32_t)ar;  // -1 at vertices that started in the tree
            if (co) co[v] = (uint32_t)(ar >> 32);
        }
    } else {
        // parent and degree into each vertex's tree record; its volume word starts at deg(v)
        const size_t row = rp.rows ? (size_t)rp.rows[idx] : (size_t)idx;
        bool bad = false;
        for (int b = 0; b < g.n; b += WAVE * NBS) {
            int32_t p[NBS];
#pragma unroll
            for (int k = 0; k < NBS; ++k) {
                const int v = b + k * WAVE + lane;
                p[k] = -1;
                if (v < g.n && v != g.root)
                    p[k] = (rp.mode != RUN_ESTIMATE) ? rp.parents_in[row * n + v]
                                                     : (int32_t)(uint32_t)aload(&sp.ws.arrow[v]);
            }
#pragma unroll
            for (int k = 0; k < NBS; ++k) {
                const int v = b + k * WAVE + lane;
                if (v >= g.n) continue;
                if (v != g.root && (p[k] < 0 || p[k] >= g.n || p[k] == v)) { bad = true; p[k] = g.root; }
                const uint64_t d = degree(g, v);
                astore(&sp.rec[2 * (size_t)v], d);
                astore(&sp.rec[2 * (size_t)v + 1], (uint64_t)(uint32_t)p[k] | (d << 32));
            }
        }
        fence_wg();
        bool ok = tree_numbering(g, sp);
        if (__ballot(bad) != 0ull) ok = false;
        int64_t f = 0;
        if constexpr (CROSS) {
            f = ok ? crossing_edges(g, sp, rp, (int32_t)row, idx) : 0;
        } else {
            if (rp.mode == RUN_CURRENT) f = path_current(sp, rp.path, rp.path_len);
            else if (rp.traversal == 2) f = f_sweep(g, sp, fen_len, lds.sweep);
            else f = f_walk(g, sp);
        }
        if (!ok) report_error(rp.ctl, DEV_BADTREE, idx);
        if (lane == 0) rp.f_out[idx] = f;
    }
    if (rp.steps_out && lane == 0) rp.steps_out[idx] = steps;
    if (rp.iters_out && lane == 0) rp.iters_out[idx] = iters;
    return true;
}

// The next work item for the calling workgroup (one atomic per workgroup).
__device__ __forceinline__ int next_item(int32_t *ctl) {
    int idx = 0;
    if (threadIdx.x == 0) idx = __hip_atomic_fetch_add(&ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // lane 0 is the first active lane: the index becomes a wave-uniform (scalar) value
    return __builtin_amdgcn_readfirstlane(idx);
}
__device__ __forceinline__ bool stopped(const int32_t *ctl) {
    return __hip_atomic_load(const_cast<int32_t *>(&ctl[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Waves per SIMD the kernel is built to fit: three at 1,024 chains (168 VGPRs;
// the LDS then allows ten workgroups per CU), two at 2,048 (LDS allows five).
template <int CH>
constexpr int waves_per_simd() { return CH <= 1024 ? 3 : 2; }

template <int CH, bool CROSS = false, bool LEAN = false>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(waves_per_simd<CH>())))
persistent_kernel(GraphDev g, SlotDev sd, RunParams rp) {
    __shared__ KernelShared<CH> lds;
    const SlotPtrs sp = slot_ptrs(sd, (size_t)g.n);
    int64_t done = 0;
    while (true) {
        const int idx = next_item(rp.ctl);
        if (idx >= rp.count || stopped(rp.ctl)) break;
        if (!process_one<CH, CROSS, LEAN>(g, sp, lds, rp, sd.fen_len, idx, (uint64_t)(rp.first + idx))) break;
        // samples finished by this workgroup, for a host that watches a long batch
        ++done;
        if (rp.progress && threadIdx.x == 0)
            __hip_atomic_store(&rp.progress[blockIdx.x], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// One persistent launch over the samples of several graphs (a batch): work
// item idx belongs to the job j with base[j] <= idx < base[j + 1], and is
// sample first[j] + launch * count[j] + (idx - base[j]) of that job's graph,
// where `launch` counts the launches of the batch so far (read from device
// memory, advanced by advance_kernel after each launch).  Every item's f,
// draws and rounds go to position idx of the batch arrays.
template <int CH, bool LEAN>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(waves_per_simd<CH>())))
batch_kernel(BatchArgs a, SlotDev sd, int32_t *ctl,
                                                     const int64_t *launch) {
    __shared__ KernelShared<CH> lds;
    const SlotPtrs sp = slot_ptrs(sd, (size_t)sd.stride);
    const int64_t L = *launch;
    while (true) {
        const int idx = next_item(ctl);
        if (idx >= a.base[a.k] || stopped(ctl)) break;
        int j = 0;
        while (j + 1 < a.k && idx >= a.base[j + 1]) ++j;
        const BatchJob &job = a.job[j];
        RunParams rp{};
        rp.seed = job.seed;
        rp.mode = RUN_ESTIMATE;
        rp.walkers = job.walkers;
        rp.traversal = job.traversal;
        rp.iter_cap = job.iter_cap;
        rp.ctl = ctl;
        rp.f_out = a.f;
        rp.steps_out = a.steps;
        rp.iters_out = a.iters;
        const uint64_t s = (uint64_t)(job.first + L * (int64_t)(a.base[j + 1] - a.base[j]) + (idx - a.base[j]));
        if (!process_one<CH, false, LEAN>(job.g, sp, lds, rp, job.g.two_m + 2, idx, s)) break;
    }
}

// Launch counter of a batch: one more launch done; the status word is cleared
// by the next launch's reset.
__global__ void advance_kernel(int64_t *launch) {
    if (threadIdx.x == 0) *launch += 1;
}

// Resident trees that contain one of the deleted edges {u, v} (as u -> v or
// v -> u in the parent array): flags[t] = 1.  One thread per (tree, edge).
__global__ void flag_trees_kernel(const int32_t *par, int32_t count, int64_t n, const int32_t *eu,
                                  const int32_t *ev, int32_t ne, uint8_t *flags) {
    const int64_t total = (int64_t)count * ne;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / ne;
        const int k = (int)(i - t * ne);
        const int32_t u = eu[k], v = ev[k];
        const int32_t *row = par + t * n;
        if (row[u] == v || row[v] == u) flags[t] = 1;
    }
}

// Trees drawn with u and v in the tree from the start (a two-tree forest
// rooted at u and v): add the edge v -> u, then re-orient the path from r so
// that every vertex points toward r.  One thread per tree.
__global__ void reroot_kernel(int32_t *par, int32_t count, int64_t n, int32_t u, int32_t v, int32_t r) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int32_t *row = par + (int64_t)t * n;
    row[v] = u;
    int32_t prev = -1, x = r;
    for (int64_t guard = 0; x != -1 && guard <= n; ++guard) {
        const int32_t nx = row[x];
        row[x] = prev;
        prev = x;
        x = nx;
    }
}

// link-cut (section 4.2) on resident trees rows[t]: the tree path between u
// and v (lengths su from u and sv from v up to their lowest common ancestor)
// has d = su + sv edges; d_out[t] = d.  With relink, edge number j (drawn by
// Philox on counter (slot, serial, ISM_CTR_LO, ISM_CTR_HI); edges counted
// from u upward, then from v upward) is removed and {u, v} added: the path
// from the endpoint on j's side up to the cut edge is reversed.  One thread
// per tree.
__global__ void link_cut_kernel(int32_t *par, const int32_t *rows, int32_t count, int64_t n, int32_t u,
                                int32_t v, uint64_t seed, uint32_t serial, int relink, int64_t *d_out,
                                int32_t *ctl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int32_t slot = rows[t];
    int32_t *row = par + (int64_t)slot * n;
    auto depth_of = [&](int32_t x) {
        int64_t d = 0;
        while (d <= n && row[x] != -1) {
            x = row[x];
            ++d;
        }
        return d;
    };
    int64_t du = depth_of(u), dv = depth_of(v);
    if (du > n || dv > n) {
        report_error(ctl, DEV_BADTREE, t);
        return;
    }
    int32_t x = u, y = v;
    int64_t su = 0, sv = 0;
    for (; du > dv; --du, ++su) x = row[x];
    for (; dv > du; --dv, ++sv) y = row[y];
    for (; x != y; ++su, ++sv) {
        x = row[x];
        y = row[y];
    }
    const int64_t d = su + sv;
    d_out[t] = d;
    if (!relink) return;
    if (d <= 0) {
        report_error(ctl, DEV_BADTREE, t);
        return;
    }
    const int64_t j = arrow_slot(seed, ((uint64_t)ISM_CTR_HI << 32) | ISM_CTR_LO, serial, (uint32_t)slot,
                                 (uint32_t)d);
    const bool u_side = j < su;
    int32_t prev = u_side ? v : u, z = u_side ? u : v;
    const int64_t steps = u_side ? j : j - su;
    for (int64_t i = 0; i <= steps; ++i) {
        const int32_t nz = row[z];
        row[z] = prev;
        prev = z;
        z = nz;
    }
}

__global__ void reset_ctl_kernel(int32_t *ctl) {
    if (threadIdx.x < 4) ctl[threadIdx.x] = 0;
}

__global__ void zero_i64_kernel(int64_t *p, int64_t len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Exact sums of f and f^2 (128-bit) and of the draw counts of items
// base[b] .. base[b+1]-1 into out[b], one block b per range (a single range:
// base = {0, count}).
struct Ranges {
    int32_t base[BATCH_MAX + 1];
};

__global__ void __launch_bounds__(256) reduce_kernel(const int64_t *f, const int64_t *steps,
                                                     const int64_t *iters, Ranges r, ReduceOut *outs) {
    const int32_t lo = r.base[blockIdx.x], count = r.base[blockIdx.x + 1] - lo;
    f += lo;
    if (steps) steps += lo;
    if (iters) iters += lo;
    ReduceOut *out = outs + blockIdx.x;
    __shared__ unsigned __int128 sh_s[256];
    __shared__ unsigned __int128 sh_q[256];
    __shared__ int64_t sh_t[256];
    __shared__ int64_t sh_i[256];
    unsigned __int128 s = 0, q = 0;
    int64_t t = 0, it = 0;
    for (int i = threadIdx.x; i < count; i += 256) {
        const __int128 x = f[i];
        s += (unsigned __int128)x;
        q += (unsigned __int128)(x * x);
        if (steps) t += steps[i];
        if (iters) it += iters[i];
    }
    sh_s[threadIdx.x] = s;
    sh_q[threadIdx.x] = q;
    sh_t[threadIdx.x] = t;
    sh_i[threadIdx.x] = it;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh_s[threadIdx.x] += sh_s[threadIdx.x + w];
            sh_q[threadIdx.x] += sh_q[threadIdx.x + w];
            sh_t[threadIdx.x] += sh_t[threadIdx.x + w];
            sh_i[threadIdx.x] += sh_i[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out->sum_lo = (uint64_t)sh_s[0];
        out->sum_hi = (int64_t)(uint64_t)(sh_s[0] >> 64);
        out->sq_lo = (uint64_t)sh_q[0];
        out->sq_hi = (uint64_t)(sh_q[0] >> 64);
        out->steps = sh_t[0];
        out->iters = sh_i[0];
    }
}

}  // namespace

hipError_t launch_reset_ctl(int32_t *ctl, hipStream_t stream) {
    hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(64), 0, stream, ctl);
    return hipGetLastError();
}

bool valid_chains(int chains) {
#define KC_CASE(C) if (chains == C) return true;
    KC_CHAIN_VARIANTS(KC_CASE)
#undef KC_CASE
    return false;
}

hipError_t launch_persistent(const GraphDev &g, const SlotDev &s, const RunParams &rp, int chains,
                             int slots, hipStream_t stream) {
    if (rp.mode == RUN_CROSS) {
        hipLaunchKernelGGL((persistent_kernel<1024, true>), dim3(slots), dim3(WAVE), 0, stream, g, s, rp);
        return hipGetLastError();
    }
#define KC_CASE(C)                                                                                   \
    if (chains == C) {                                                                              \
        if (rp.lean)                                                                                \
            hipLaunchKernelGGL((persistent_kernel<C, false, true>), dim3(slots), dim3(WAVE), 0, stream, g, s, rp); \
        else                                                                                        \
            hipLaunchKernelGGL((persistent_kernel<C, false, false>), dim3(slots), dim3(WAVE), 0, stream, g, s, rp); \
        return hipGetLastError();                                                                   \
    }
    KC_CHAIN_VARIANTS(KC_CASE)
#undef KC_CASE
    return hipErrorInvalidValue;
}

int sampler_chains() { return MAX_CHAINS; }

int batch_blocks_per_cu(int chains) {
    int blocks = 0;
#define KC_CASE(C)                                                                                   \
    if (chains == C) {                                                                              \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel<C, false>, WAVE, 0) != \
            hipSuccess)                                                                             \
            return 0;                                                                               \
        return blocks;                                                                              \
    }
    KC_CHAIN_VARIANTS(KC_CASE)
#undef KC_CASE
    return 0;
}

int persistent_blocks_per_cu(int chains) {
    int blocks = 0;
#define KC_CASE(C)                                                                                   \
    if (chains == C) {                                                                              \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, persistent_kernel<C>, WAVE, 0) !=   \
            hipSuccess)                                                                             \
            return 0;                                                                               \
        return blocks;                                                                              \
    }
    KC_CHAIN_VARIANTS(KC_CASE)
#undef KC_CASE
    return 0;
}

hipError_t launch_reduce(const int64_t *f, const int64_t *steps, const int64_t *iters, int32_t count,
                         ReduceOut *out, hipStream_t stream) {
    Ranges r{};
    r.base[0] = 0;
    r.base[1] = count;
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, stream, f, steps, iters, r, out);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs &a, const SlotDev &s, int32_t *ctl, int64_t *launch, ReduceOut *out,
                        int chains, int slots, hipStream_t stream) {
    if (a.k < 1 || a.k > BATCH_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(64), 0, stream, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // lean looks when every job of the batch takes them
    bool lean = true;
    for (int j = 0; j < a.k; ++j) lean = lean && a.job[j].lean != 0;
#define KC_CASE(C)                                                                                \
    if (chains == C) {                                                                           \
        if (lean)                                                                                \
            hipLaunchKernelGGL((batch_kernel<C, true>), dim3(slots), dim3(WAVE), 0, stream, a, s, ctl, launch); \
        else                                                                                     \
            hipLaunchKernelGGL((batch_kernel<C, false>), dim3(slots), dim3(WAVE), 0, stream, a, s, ctl, launch); \
        e = hipGetLastError();                                                                   \
    }
    e = hipErrorInvalidValue;
    KC_CHAIN_VARIANTS(KC_CASE)
#undef KC_CASE
    if (e != hipSuccess) return e;
    Ranges r{};
    for (int j = 0; j <= a.k; ++j) r.base[j] = a.base[j];
    hipLaunchKernelGGL(reduce_kernel, dim3(a.k), dim3(256), 0, stream, a.f, a.steps, a.iters, r, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, stream, launch);
    return hipGetLastError();
}

hipError_t launch_reroot(int32_t *par, int32_t count, int64_t n, int32_t u, int32_t v, int32_t r,
                         hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(reroot_kernel, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, stream, par, count, n,
                       u, v, r);
    return hipGetLastError();
}

hipError_t launch_link_cut(int32_t *par, const int32_t *rows, int32_t count, int64_t n, int32_t u, int32_t v,
                           uint64_t seed, uint32_t serial, int relink, int64_t *d_out, int32_t *ctl,
                           hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(link_cut_kernel, dim3((count + 63) / 64), dim3(64), 0, stream, par, rows, count, n, u, v,
                       seed, serial, relink, d_out, ctl);
    return hipGetLastError();
}

hipError_t launch_flag_trees(const int32_t *par, int32_t count, int64_t n, const int32_t *eu,
                             const int32_t *ev, int32_t ne, uint8_t *flags, hipStream_t stream) {
    const int64_t total = (int64_t)count * ne;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(flag_trees_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, par, count, n, eu, ev,
                       ne, flags);
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int64_t len, hipStream_t stream) {
    if (len <= 0) return hipSuccess;
    int64_t blocks = (len + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_i64_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, len);
    return hipGetLastError();
}

}  // namespace kc
