// tqr: tiled QR (Buttari, Langou, Kurzak, Dongarra) on one MI355X.
//
// Implementation header shared by the library's translation units: the
// scheduler, the four tile kernels of Sec. 3.1 as workgroup tasks, the
// persistent task-graph scheduler of Sec. 3.3, and the host-side templates
// that launch them.  Every (tile_b, inner_ib) pair is instantiated in a
// translation unit of its own (tqr_inst.hip), so that the pairs compile in
// parallel; tqr.hip holds the C entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "tqr.h"
#include "tqr_device.h"
#include "tqr_graph.h"

namespace tqr {

// ===========================================================================
// Layout: column-major <-> tiles (Block Data Layout, Sec. 3.4)
// ===========================================================================
// Tile (i,j) of a p-row grid of b x tw tiles starts at ((j*p)+i)*b*tw.
// (defined in tqr.hip)
__global__ void k_cm_to_tiles(const double *__restrict__ A, int64_t lda, int64_t m, int64_t n,
                              double *__restrict__ W, int p, int b, int tw);
__global__ void k_tiles_to_cm(const double *__restrict__ W, int p, int b, int tw, double *__restrict__ A,
                              int64_t lda, int64_t m, int64_t n);

// ===========================================================================
// Scheduler state (in the caller's workspace)
// ===========================================================================
// Hot words are grouped by who touches them, each group in its own 256-byte
// block: the done count and status; the queue words; the idle-worker bitmap.
// Every worker also owns a mailbox on a 128-byte line of its own, the only
// word it polls while idle.
constexpr int kMaxWorkers = 2048;      // persistent workgroups per launch, at most
constexpr int kMboxStride = 32;        // ints between mailboxes
constexpr int32_t kMboxEmpty = -1;     // mailbox values; task ids are >= 0
constexpr int32_t kMboxWake = -2;      // look at the ready queues again
constexpr int32_t kMboxStop = -3;      // the graph is finished or aborted: exit

struct SchedState {
    uint32_t pad_a;
    uint32_t done;    // number of finished tasks without successors
    int32_t status;   // 0, or TQR_EABORTED
    uint32_t nsinks;  // number of tasks without successors (set by k_sched_seed)
    int32_t panel;    // factorisation: GEQRT tasks started so far (priority reference)
    uint32_t pad0[59];
    uint64_t ht[8];   // per priority level: (tail << 32) | head of its queue
    uint32_t pad1[48];
    uint64_t idle[kMaxWorkers / 64];  // bit w set: worker w waits on its mailbox
};
static_assert(sizeof(SchedState) == 768, "state layout");
static_assert(offsetof(SchedState, ht) == 256 && offsetof(SchedState, idle) == 512, "hot words in their own blocks");

struct Sched {
    SchedState *st;
    int32_t *mbox;    // kMaxWorkers mailboxes, kMboxStride ints apart
    int32_t *cnt;     // remaining in-degree per task
    int32_t *queue;   // kLevels arrays of `cap` task ids, -1 = not yet written
    int64_t cap;      // = number of tasks
    int64_t ntasks;
};

constexpr int64_t kMboxBytes = (int64_t)kMaxWorkers * kMboxStride * 4;

__host__ __device__ inline int64_t sched_bytes(int64_t ntasks) {
    return (int64_t)sizeof(SchedState) + kMboxBytes + ((ntasks * 4 * (1 + kLevels) + 255) / 256) * 256;
}

__host__ inline Sched sched_at(void *base, int64_t ntasks) {
    Sched s;
    char *c = reinterpret_cast<char *>(base);
    s.st = reinterpret_cast<SchedState *>(c);
    s.mbox = reinterpret_cast<int32_t *>(c + sizeof(SchedState));
    s.cnt = reinterpret_cast<int32_t *>(c + sizeof(SchedState) + kMboxBytes);
    s.queue = s.cnt + ntasks;
    s.cap = ntasks;
    s.ntasks = ntasks;
    return s;
}

// Grid: max(ntasks, kMaxWorkers) threads.
template <class G>
__global__ void k_sched_init(G g, Sched s) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < s.ntasks) {
        s.cnt[t] = g.indegree(g.decode(t));
        for (int l = 0; l < kLevels; ++l) s.queue[l * s.cap + t] = -1;
    }
    if (t < kMaxWorkers) s.mbox[t * kMboxStride] = kMboxEmpty;
    if (t < kMaxWorkers / 64) s.st->idle[t] = 0;
    if (t == 0) {
        for (int l = 0; l < 8; ++l) s.st->ht[l] = 0;
        s.st->done = 0;
        s.st->status = 0;
        s.st->nsinks = 0;
        s.st->panel = 0;
    }
}

template <class G>
__device__ __host__ inline int level_of(const G &, const Task &, int, int = 0) { return 0; }
template <>
__device__ __host__ inline int level_of<FactorGraph>(const FactorGraph &g, const Task &t, int policy, int panel) {
    return g.level(t, policy, panel);
}
template <>
__device__ __host__ inline int level_of<TrsmGraph>(const TrsmGraph &, const Task &t, int, int) {
    return t.kind == 0 ? 0 : 1;
}

// Scheduler words (queue words and slots, dependency counters, the idle
// bitmap, mailboxes, the done count and the status) are accessed with relaxed
// system-scope atomics, which no XCD serves from a stale copy in its own L2.
// Tile data is ordered by explicit fences: a task releases its writes before
// it decrements its successors' counters (each wave waits for its own stores,
// then thread 0 issues one agent-scope release, which writes the XCD's L2
// back), and every task acquires (thread 0, agent-scope acquire: an L2
// invalidate) before its body runs, wherever it was taken from.  On this
// chip these cache operations are costly and act on the whole L2, so each
// task issues exactly one of each.
#define TQR_FLAG_SCOPE __HIP_MEMORY_SCOPE_SYSTEM

__device__ __forceinline__ uint64_t rt_clock() { return wall_clock64(); }

template <class T>
__device__ __forceinline__ T flag_load(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

__device__ __forceinline__ void set_status(const Sched &s, int32_t v) {
    __hip_atomic_store(&s.st->status, v, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

// Pushes the tasks without predecessors and counts the tasks without
// successors.  Runs as its own launch after k_sched_init, so every slot and
// count is already cleared; the persistent launch comes after it.
template <class G>
__global__ void k_sched_seed(G g, Sched s, int policy) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.ntasks) return;
    const Task task = g.decode(t);
    if (g.num_successors(task) == 0) __hip_atomic_fetch_add(&s.st->nsinks, 1u, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
    if (g.indegree(task) != 0) return;
    const int lvl = level_of(g, task, policy);
    const uint32_t pos = (uint32_t)(__hip_atomic_fetch_add(&s.st->ht[lvl], 1ull << 32, __ATOMIC_RELAXED, TQR_FLAG_SCOPE) >> 32);
    __hip_atomic_store(&s.queue[lvl * s.cap + pos], (int32_t)t, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

constexpr uint32_t kMaxSpins = 1u << 26;  // a second bound on every wait, independent of the clock

// Writes kMboxStop into every worker's mailbox.
__device__ void broadcast_stop(const Sched &s, int nworkers) {
    for (int w = 0; w < nworkers; ++w)
        __hip_atomic_store(&s.mbox[w * kMboxStride], kMboxStop, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

__device__ void abort_run(const Sched &s, int nworkers) {
    set_status(s, TQR_EABORTED);
    broadcast_stop(s, nworkers);
}

// Far-first workers (RunOpts::far_every): under the column policy one worker
// in far_every serves the update levels farthest column first, so that work
// for the columns the panels reach later keeps moving even while nearer
// levels never run dry, instead of piling up in the last level and holding
// up a panel when its column comes near.  Measured on the square
// factorisation (one worker in four); on tall grids, where the chains of
// TSQRT tasks pace the run, they slow it down and are not used.
constexpr int kFarEverySquare = 4;

// One look at the ready queues: takes the head task of the highest-priority
// non-empty level (for a far-first worker, levels 2.. in reverse).  Returns
// the task id, -1 if every level looked empty or other workers took what
// there was, -2 after an abort.
__device__ int32_t try_pop(const Sched &s, bool far_first, uint64_t deadline, uint32_t &spins, int nworkers) {
    uint64_t w[kLevels];
#pragma unroll
    for (int l = 0; l < kLevels; ++l) w[l] = flag_load(&s.st->ht[l]);
    for (int r = 0; r < kLevels; ++r) {
        const int l = far_first && r >= 2 ? kLevels + 1 - r : r;
        uint64_t cur = w[l];
        // a failed exchange returns the current word: retry at once while
        // the level still holds work (a push also changes the word)
        for (int tries = 0; tries < 4 && (uint32_t)cur < (uint32_t)(cur >> 32); ++tries) {
            if (__hip_atomic_compare_exchange_strong(&s.st->ht[l], &cur, cur + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     TQR_FLAG_SCOPE)) {
                // the pusher reserves a slot before it writes the task id, so
                // the slot may still read -1 for a moment
                const int32_t *slot = &s.queue[l * s.cap + (uint32_t)cur];
                int32_t v;
                while ((v = flag_load(slot)) < 0) {
                    if (rt_clock() > deadline || ++spins > kMaxSpins) {
                        abort_run(s, nworkers);
                        return -2;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                return v;
            }
        }
    }
    return -1;
}

// Every level's word is loaded before any is looked at: one memory round
// trip instead of one per level (read_queue_words), issued early by the
// caller so that the trip overlaps other waits.
__device__ __forceinline__ void read_queue_words(const Sched &s, uint64_t (&w)[kLevels]) {
#pragma unroll
    for (int l = 0; l < kLevels; ++l) w[l] = flag_load(&s.st->ht[l]);
}
__device__ __forceinline__ bool queue_has_level_below(const uint64_t (&w)[kLevels], int lvl) {
    bool any = false;
#pragma unroll
    for (int l = 0; l < kLevels; ++l) any |= l < lvl && (uint32_t)w[l] < (uint32_t)(w[l] >> 32);
    return any;
}

__device__ __forceinline__ void push_one(const Sched &s, int lvl, int32_t t) {
    const uint32_t pos = (uint32_t)(__hip_atomic_fetch_add(&s.st->ht[lvl], 1ull << 32, __ATOMIC_RELAXED, TQR_FLAG_SCOPE) >> 32);
    __hip_atomic_store(&s.queue[lvl * s.cap + pos], t, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

__device__ void wake_idle(const Sched &s, int count, int nworkers);

// Clears this worker's idle bit.  Returns kMboxEmpty when the bit was still
// set.  Otherwise another worker claimed this one first and is writing its
// mailbox: the message (a task id, kMboxWake or kMboxStop) is waited for,
// taken out and returned.
__device__ int32_t withdraw_idle(const Sched &s, uint64_t *word, uint64_t bit, int32_t *mb, uint64_t deadline,
                                 uint32_t &spins, int nworkers) {
    const uint64_t old = __hip_atomic_fetch_and(word, ~bit, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
    if (old & bit) return kMboxEmpty;
    while (flag_load(mb) == kMboxEmpty) {
        if (rt_clock() > deadline || ++spins > kMaxSpins) {
            abort_run(s, nworkers);
            return kMboxStop;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return __hip_atomic_exchange(mb, kMboxEmpty, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}

// Thread 0 of an idle worker: returns the next task, or -1 when the graph is
// finished or aborted.  An idle worker sets its bit in the idle bitmap, looks
// at the queues once more, and then polls only its own mailbox, where a
// worker that releases tasks either hands one over directly (its id) or
// leaves a wake-up (look at the queues).  A worker that publishes tasks
// hands them to claimed idle workers or pushes them and then wakes idle
// workers; with a store-load fence between the write and the read on both
// sides (bit set -> queue look; push -> bitmap look), a task published while
// a worker goes idle is seen by one of the two, so no task is left in a
// queue while every worker waits.  A sleeping worker also looks at
// the queues every 64 polls (a queue word can be contended enough that a
// woken worker loses every exchange for a while).  Waits are bounded by the
// deadline and a spin count; the periodic check of the done count, the
// status and the abort flag also ends a wait.
// Store-load fence for scheduler words: they are accessed only with
// system-scope atomics, which are performed at memory and never served from
// an L2, so waiting until this wave's earlier accesses are complete orders
// them before its later ones (no L2 writeback or invalidate, which an
// agent-scope fence would issue on the whole XCD's L2).  The signal fences
// keep the compiler from moving memory accesses across the wait.
__device__ __forceinline__ void sched_store_load_fence() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <class G>
__device__ int32_t idle_wait(const G &g, int policy, int far_every, const Sched &s, uint32_t nsinks,
                             const volatile int32_t *abort_flag, uint64_t deadline, int me, int nworkers) {
    uint32_t spins = 0;
    uint64_t *word = &s.st->idle[me >> 6];
    const uint64_t bit = 1ull << (me & 63);
    int32_t *mb = &s.mbox[me * kMboxStride];
    const bool far_first = far_every > 0 && me % far_every == far_every - 1;
    for (;;) {
        if (flag_load(&s.st->status) != 0) return -1;
        int32_t t = try_pop(s, far_first, deadline, spins, nworkers);
        if (t >= 0) return t;
        if (t == -2) return -1;
        __hip_atomic_fetch_or(word, bit, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
        sched_store_load_fence();
        t = try_pop(s, far_first, deadline, spins, nworkers);
        if (t >= 0) {
            const int32_t m = withdraw_idle(s, word, bit, mb, deadline, spins, nworkers);
            if (m >= 0) {
                // a task handed over while this worker took one itself goes
                // back to the queues
                push_one(s, level_of(g, g.decode(m), policy), m);
                wake_idle(s, 1, nworkers);
            } else if (m == kMboxStop) {
                __hip_atomic_store(mb, kMboxStop, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            }
            return t;
        }
        if (t == -2) return -1;
        uint32_t polls = 0;
        for (;;) {
            if (flag_load(mb) != kMboxEmpty) {
                const int32_t v = __hip_atomic_exchange(mb, kMboxEmpty, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
                if (v == kMboxStop) return -1;
                if (v >= 0) return v;        // handed over
                if (v != kMboxEmpty) break;  // woken: look at the queues
            }
            if ((++polls & 63) == 0) {
                if (flag_load(&s.st->done) >= nsinks || flag_load(&s.st->status) != 0) return -1;
                if ((abort_flag && flag_load(const_cast<const int32_t *>(abort_flag))) || rt_clock() > deadline) {
                    abort_run(s, nworkers);
                    return -1;
                }
                uint64_t qw[kLevels];
                read_queue_words(s, qw);
                if (queue_has_level_below(qw, kLevels)) {
                    const int32_t m = withdraw_idle(s, word, bit, mb, deadline, spins, nworkers);
                    if (m >= 0) return m;
                    if (m == kMboxStop) return -1;
                    break;
                }
            }
            if (++spins > kMaxSpins) {
                abort_run(s, nworkers);
                return -1;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
}

// Thread 0 with ready tasks to publish (ready[r] for the r with lvl[r] >= 0,
// taken in level order): claims idle workers in the bitmap and writes one
// task id into each one's mailbox; a handed-over task gets lvl[r] = -1.  A
// mailbox that is not empty (a message not yet taken) keeps its task for the
// queues.  Returns the number handed over.
__device__ int handoff_ready(const Sched &s, const int32_t *ready, int8_t *lvl, int nr, int nworkers) {
    int left = 0;
    for (int r = 0; r < nr; ++r) left += lvl[r] >= 0;
    if (left == 0) return 0;
    sched_store_load_fence();
    int handed = 0, cur_lvl = 0, cur_r = 0;
    // next task in priority order (level, then position); -1 when none left
    auto next_task = [&]() -> int {
        for (; cur_lvl < kLevels; ++cur_lvl, cur_r = 0)
            for (; cur_r < nr; ++cur_r)
                if (lvl[cur_r] == cur_lvl) return cur_r;
        return -1;
    };
    const int nwords = (nworkers + 63) >> 6;
    for (int wi = 0; wi < nwords && left > 0; ++wi) {
        uint64_t v = flag_load(&s.st->idle[wi]);
        while (v != 0 && left > 0) {
            uint64_t mask = 0, rest = v;
            for (int c = 0; c < left && rest != 0; ++c) {
                const uint64_t low = rest & (~rest + 1);
                mask |= low;
                rest &= rest - 1;
            }
            const uint64_t old = __hip_atomic_fetch_and(&s.st->idle[wi], ~mask, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            uint64_t got = old & mask;
            while (got != 0) {
                const int w = (wi << 6) + __builtin_ctzll(got);
                got &= got - 1;
                const int r = next_task();
                int32_t expect = kMboxEmpty;
                if (r >= 0 && __hip_atomic_compare_exchange_strong(&s.mbox[w * kMboxStride], &expect, ready[r],
                                                                   __ATOMIC_RELAXED, __ATOMIC_RELAXED, TQR_FLAG_SCOPE)) {
                    lvl[r] = -1;
                    ++handed;
                    --left;
                } else if (r < 0) {
                    // more workers claimed than tasks left (cannot happen
                    // with one claimer per word, kept for safety): wake it
                    __hip_atomic_compare_exchange_strong(&s.mbox[w * kMboxStride], &expect, kMboxWake,
                                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
                }
            }
            v = old & ~mask;
        }
    }
    return handed;
}

// Thread 0 after pushing `count` tasks: wakes up to `count` idle workers.
__device__ void wake_idle(const Sched &s, int count, int nworkers) {
    sched_store_load_fence();
    const int nwords = (nworkers + 63) >> 6;
    for (int wi = 0; wi < nwords && count > 0; ++wi) {
        uint64_t v = flag_load(&s.st->idle[wi]);
        while (v != 0 && count > 0) {
            // claim up to `count` of the set bits with one exchange
            uint64_t mask = 0, rest = v;
            for (int c = 0; c < count && rest != 0; ++c) {
                const uint64_t low = rest & (~rest + 1);
                mask |= low;
                rest &= rest - 1;
            }
            const uint64_t old = __hip_atomic_fetch_and(&s.st->idle[wi], ~mask, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            uint64_t got = old & mask;
            while (got != 0) {
                const int w = (wi << 6) + __builtin_ctzll(got);
                got &= got - 1;
                int32_t expect = kMboxEmpty;
                // never overwrite a stop
                __hip_atomic_compare_exchange_strong(&s.mbox[w * kMboxStride], &expect, kMboxWake, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
                --count;
            }
            v = old & ~mask;
        }
    }
}

__device__ __forceinline__ int xcc_id() {
    int v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xf;
}

// The hardware slot register of the wave (CU, shader array and engine ids).
__device__ __forceinline__ int hw_id() {
    int v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(v));
    return v;
}

// Per-task trace record: taken, acquired, body done, released (device
// constant-rate clock), workgroup, XCD, hardware slot register, and 1 when
// the task ran as its predecessor's continuation (0 when it was popped).
constexpr int kTraceFields = 8;


struct RunOpts {
    int64_t *trace;
    int64_t ntrace;  // tasks with a trace record (the paper's tasks; helper tasks have none)
    const volatile int32_t *abort_flag;
    int64_t timeout;
    int policy;
    int far_every;  // 0, or one far-first worker in this many
};

// Progress of the chain of tasks that rewrite the triangle R_kk (GEQRT(k),
// then TSQRT(k+1,k), TSQRT(k+2,k), ...).  Inner block s of these tasks
// touches only row block s of R_kk (and, for the panel of block s+1 that the
// lookahead factors, the diagonal block of row block s+1), so a task of the
// chain can follow its predecessor one row block behind instead of waiting
// for it to finish: `prev` counts the row blocks of R_kk the predecessor has
// finished, `mine` the same for this task (null: nothing to wait for, or
// nobody waiting).  Waits are bounded by `deadline`; a timeout sets *status to
// TQR_EABORTED and lets the task run on (its results are then void).
struct Pipe {
    int32_t *prev, *mine, *status;
    uint64_t deadline;
    // TSQRT(i,k) and its helper: panels stored (pv), blocks the helper has
    // applied to its strips (hb), and the claim of those strips (claim: 0
    // open, 1 the TSQRT kept them, 2 the helper took them); null without a
    // helper
    int32_t *pv = nullptr, *hb = nullptr, *claim = nullptr;
    // the predecessor TSQRT's helper words (row block s of R_kk is final
    // when the predecessor has finished it and, if its helper took strips,
    // the helper has applied block s)
    int32_t *prev_hb = nullptr, *prev_claim = nullptr;
};

constexpr uint64_t kClaimTicks = 2000;  // how long a TSQRT waits for its helper (device clock ticks)

// Thread 0: waits until the predecessor has finished `target` row blocks,
// then acquires its writes.
__device__ void pipe_wait_on(const Pipe &pp, const int32_t *word, int target) {
    uint32_t n = 0;
    while (flag_load(word) < target) {
        if (flag_load(pp.status) != 0) return;
        if (rt_clock() > pp.deadline || ++n > kMaxSpins) {
            __hip_atomic_store(pp.status, (int32_t)TQR_EABORTED, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void pipe_wait(const Pipe &pp, int target) { pipe_wait_on(pp, pp.prev, target); }

// Thread 0 of a chain task: waits until row blocks 0 .. rows-1 of R_kk are
// final (the predecessor's own progress, then its helper's; the claim is
// settled before the predecessor publishes anything).
__device__ void pipe_wait_rows(const Pipe &pp, int rows, int nb) {
    pipe_wait(pp, rows);
    if (pp.prev_claim && flag_load(pp.prev_claim) == 2) {
        const int t = rows < nb - 2 ? rows : nb - 2;
        if (t > 0) pipe_wait_on(pp, pp.prev_hb, t);
    }
}

// Thread 0, after a workgroup barrier (or after its own wave's stores):
// releases those writes and publishes `count`.
__device__ void pipe_publish_on(int32_t *word, int count) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(word, count, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
}
__device__ __forceinline__ void pipe_publish(const Pipe &pp, int count) { pipe_publish_on(pp.mine, count); }

// The calling wave waits until its global stores are complete (have reached
// the L2): s_waitcnt vmcnt(0), with the other counters left alone.
__device__ __forceinline__ void wait_own_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A workgroup barrier orders the waves but does not wait for their global
// stores, and thread 0's release before a publish (an L2 writeback and a
// wait for its own wave's stores) covers other waves' stores only once they
// are complete: every other wave waits for its stores before the barrier
// that precedes such a publish.
__device__ __forceinline__ void release_before_publish() {
    if (wave_id() != 0) wait_own_stores();
}

// ===========================================================================
// Tile kernels (bodies run by one workgroup)
// ===========================================================================
template <int B, int IB>
struct TileKernels {
    static constexpr int NB = B / IB;
    static constexpr int WCOLS = 16 * NWAVES;              // columns per workgroup pass
    static constexpr int LDP = IB + B + 1;                  // panel leading dimension (odd: LDS banks)
    static constexpr int LDV = B + 1;                       // staged V leading dimension
    static constexpr size_t PANEL_DOUBLES = (size_t)LDP * IB;
    static constexpr size_t LDS_GENERIC = (PANEL_DOUBLES + 2 * IB * IB + 2 * IB + NWAVES) * sizeof(double);
    // ib = 16 panels: two V buffers (16 x LDV), two T buffers (16 x 16), the
    // 16 x 16 diagonal block of R for TSQRT, the one-wave panel scratch
    // ... and two strip handoff buffers (a strip in the register layout of
    // Strip<B>: B/16 row blocks of 64 lanes x 4 doubles)
    static constexpr size_t HAND_OFFSET = 2 * 16 * (size_t)LDV + 2 * 256 + 256 + kPanelScratch;
    static constexpr size_t HAND_DOUBLES = (size_t)(B / 16) * 256;
    static constexpr size_t LDS_IB16 = (HAND_OFFSET + 2 * HAND_DOUBLES) * sizeof(double);
    // LARFB/SSRFB with ib = 16 stage V and T of the next inner block while
    // the current one is applied: two buffers of (LDV x 16 + 16 x 16)
    static constexpr size_t STAGE_DOUBLES = (size_t)LDV * IB + IB * IB;
    static constexpr bool DBUF = IB == 16;
    static constexpr size_t LDS_DBUF = DBUF ? 2 * STAGE_DOUBLES * sizeof(double) : 0;
    static constexpr size_t LDS_MAX1 = IB == 16 && LDS_IB16 > LDS_GENERIC ? LDS_IB16 : LDS_GENERIC;
    static constexpr size_t LDS_BYTES = LDS_DBUF > LDS_MAX1 ? LDS_DBUF : LDS_MAX1;
    static constexpr int STAGE_V = B * IB / NT;               // V doubles per thread per block
    static constexpr int STAGE_T = (IB * IB + NT - 1) / NT;   // T doubles per thread per block
    static constexpr int RPL = B >= 64 ? B / 64 : 1;        // panel rows per lane (one-wave panels)
    static constexpr int PU = 4;                            // column steps unrolled per group in the panels

    // A strip into LDS as Vl[c * LDV + r].
    __device__ __forceinline__ static void strip_to_lds(const Strip<B> &C, double *Vl) {
        const int l = lane_id();
        double *p = Vl + (l & 15) * LDV + 4 * (l >> 4);
#pragma unroll
        for (int rb = 0; rb < B / 16; ++rb) {
            p[16 * rb] = C.v[rb].x;
            p[16 * rb + 1] = C.v[rb].y;
            p[16 * rb + 2] = C.v[rb].z;
            p[16 * rb + 3] = C.v[rb].w;
        }
    }

    // Handoff buffer of strip j (alternating by j).  In block s of GEQRT and
    // TSQRT the wave that applies the block to strip s+2, the next panel but
    // one, leaves it here instead of in memory; the lookahead of that panel
    // in block s+1 takes it from here.
    __device__ __forceinline__ static double *hand(double *smem, int j) {
        return smem + HAND_OFFSET + (size_t)(j & 1) * HAND_DOUBLES;
    }
    __device__ __forceinline__ static void strip_to_hand(const Strip<B> &C, double *H) {
        d4 *p = reinterpret_cast<d4 *>(H) + lane_id();
#pragma unroll
        for (int rb = 0; rb < B / 16; ++rb) p[64 * rb] = C.v[rb];
    }
    __device__ __forceinline__ static void hand_to_strip(Strip<B> &C, const double *H) {
        const d4 *p = reinterpret_cast<const d4 *>(H) + lane_id();
#pragma unroll
        for (int rb = 0; rb < B / 16; ++rb) C.v[rb] = p[64 * rb];
    }

    // Row block rb (rows 16rb .. 16rb+15) of a strip to global memory.
    __device__ __forceinline__ static void strip_store_block(const Strip<B> &C, double *col0, int rb) {
        const int l = lane_id();
        d4 *p = reinterpret_cast<d4 *>(col0 + (size_t)(l & 15) * B + 4 * (l >> 4) + 16 * rb);
#pragma unroll
        for (int r = 0; r < B / 16; ++r)
            if (r == rb) *p = C.v[r];
    }

    // GEQRT with ib = 16.  Wave 0 factors the panels one after another, each
    // in its registers (ge_panel16); before factoring panel j it applies block
    // j-1 to it (lookahead), while waves 1..3 apply block j-1 to the columns
    // right of panel j on the matrix cores.  V and T of the last factored
    // block alternate between two LDS buffers; one barrier per block.
    __device__ __forceinline__ static void geqrt16(double *Akk, double *Tkk, double *Vkk, double *smem, const Pipe &pp) {
        // buffer x & 1 by arithmetic on smem (not a pointer array) so that
        // the compiler keeps these LDS addresses and emits LDS instructions
        auto Vb = [smem](int x) { return smem + (x & 1) * (16 * LDV); };
        auto Tb = [smem](int x) { return smem + 32 * LDV + (x & 1) * 256; };
        double *Pl = smem + 32 * LDV + 512 + 256;
        const int w = __builtin_amdgcn_readfirstlane(wave_id());
        const bool t0 = threadIdx.x == 0;
        if (w == 0) geqrt16_panel(Akk, Tkk, Vkk, 0, nullptr, nullptr, Vb(0), Tb(0), Pl, nullptr);
        __syncthreads();
        if (NB == 1 && pp.mine && t0) pipe_publish(pp, 1);
#pragma unroll 1
        for (int s = 0; s + 1 < NB; ++s) {
            double *Vs = Vb(s & 1), *Ts = Tb(s & 1);
            if (w == 0) {
                geqrt16_panel(Akk, Tkk, Vkk, s + 1, Vs, Ts, Vb((s + 1) & 1), Tb((s + 1) & 1), Pl,
                              s + 1 >= 2 ? hand(smem, s + 1) : nullptr);
            } else {
                for (int j = s + 1 + w; j < NB; j += NWAVES - 1) {
                    Strip<B> C;
                    strip_load<B>(C, Akk + (size_t)16 * j * B, B);
                    panel_update<B, 16, true, false>(C, nullptr, Vs, LDV, Ts, 16 * s);
                    if (j == s + 2) {
                        // the next panel but one: to the handoff buffer, and
                        // only its final row block s to memory (the panel
                        // writes the rows below)
                        strip_to_hand(C, hand(smem, j));
                        strip_store_block(C, Akk + (size_t)16 * j * B, s);
                    } else {
                        strip_store<B>(C, Akk + (size_t)16 * j * B, B, s);
                    }
                }
            }
            if (pp.mine) release_before_publish();
            __syncthreads();
            // row block s is final (and so is row block NB-1 after the last block)
            if (pp.mine && t0) pipe_publish(pp, s + 2 == NB ? NB : s + 1);
        }
    }

    // Wave 0 of geqrt16: panel j (pivot rows cj .. cj+15), after applying
    // block j-1 (Vs, Ts) to it when j > 0; V_j and T_j go to Vn and Tn (LDS)
    // and to Vkk, Tkk and the tile.
    __device__ __forceinline__ static void geqrt16_panel(double *Akk, double *Tkk, double *Vkk, int j, const double *Vs,
                                                         const double *Ts, double *Vn, double *Tn, double *Pl,
                                                         const double *H) {
        const int l = lane_id();
        const int cj = 16 * j;
        double *colj = Akk + (size_t)cj * B;
        {
            Strip<B> C;
            // the strip comes from the handoff buffer when one is given
            if (H)
                hand_to_strip(C, H);
            else
                strip_load<B>(C, colj, B);
            if (j > 0) {
                panel_update<B, 16, true, false>(C, nullptr, Vs, LDV, Ts, cj - 16);
                strip_store_block(C, colj, j - 1);  // the R rows of block j-1
            }
            strip_to_lds(C, Vn);
        }
        double x[RPL][16];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = cj + l + 64 * i;
#pragma unroll
            for (int c = 0; c < 16; ++c) x[i][c] = r < B ? Vn[c * LDV + r] : 0.0;
        }
        ge_panel16u<RPL, PU>(x, Tn, Pl);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int rr = l + 64 * i, r = cj + rr;
            if (r < B) {
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    colj[(size_t)c * B + r] = x[i][c];
                    // dense unit-lower V: zero above the pivot, one on it
                    const double vd = rr > c ? x[i][c] : (rr == c ? 1.0 : 0.0);
                    Vn[c * LDV + r] = vd;
                    Vkk[(size_t)(cj + c) * B + r] = vd;
                }
            }
        }
        for (int r = l; r < cj; r += 64) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                Vn[c * LDV + r] = 0.0;
                Vkk[(size_t)(cj + c) * B + r] = 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Tkk[(size_t)cj * 16 + l + 64 * q] = Tn[l + 64 * q];
    }

    // TSQRT with ib = 16, organised as geqrt16: wave 0 factors [R_kk block;
    // A_ik panel] pairs (ts_panel16) with lookahead, waves 1..3 apply each
    // block to the columns right of the next panel.
    // Strips [help_split(), NB) of a TSQRT go to its helper when the helper
    // claims them (about 5/16 of the strips: the helper's four waves then
    // carry as much trailing work per block as the TSQRT's three).
    __device__ __forceinline__ static int help_split() { return NB - (5 * NB) / 16; }

    __device__ __forceinline__ static void tsqrt16(double *Akk, double *Aik, double *Tik, double *smem, const Pipe &pp) {
        // buffer x & 1 by arithmetic on smem (not a pointer array) so that
        // the compiler keeps these LDS addresses and emits LDS instructions
        auto Vb = [smem](int x) { return smem + (x & 1) * (16 * LDV); };
        auto Tb = [smem](int x) { return smem + 32 * LDV + (x & 1) * 256; };
        double *Rd = smem + 32 * LDV + 512;
        const int w = __builtin_amdgcn_readfirstlane(wave_id());
        const bool t0 = threadIdx.x == 0;
        __shared__ int32_t s_split;
        // block s touches row block s of R_kk and, through the lookahead
        // panel s+1, the diagonal block of row block s+1; the predecessor
        // touches neither after its own block s, so block s may start once
        // the predecessor has published s+1 finished row blocks
        if (pp.prev) {
            if (t0) pipe_wait_rows(pp, 1, NB);
            __syncthreads();
        }
        if (w == 0) {
            tsqrt16_panel(Akk, Aik, Tik, 0, nullptr, nullptr, Vb(0), Tb(0), Rd, NB, pp, nullptr);
        } else if (w == 1 && lane_id() == 0) {
            // while panel 0 is factored, give the helper (released when this
            // task started) a moment to claim its strips; otherwise keep them
            int32_t expect = 0;
            if (pp.claim) {
                const uint64_t until = rt_clock() + kClaimTicks;
                while (flag_load(pp.claim) == 0 && rt_clock() < until) __builtin_amdgcn_s_sleep(1);
                __hip_atomic_compare_exchange_strong(pp.claim, &expect, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     TQR_FLAG_SCOPE);
            }
            s_split = expect == 2 ? help_split() : NB;
        }
        __syncthreads();
        const int split = __builtin_amdgcn_readfirstlane(s_split);
        if (NB == 1 && pp.mine && t0) pipe_publish(pp, 1);
#pragma unroll 1
        for (int s = 0; s + 1 < NB; ++s) {
            double *Vs = Vb(s & 1), *Ts = Tb(s & 1);
            if (w == 0) {
                tsqrt16_panel(Akk, Aik, Tik, s + 1, Vs, Ts, Vb((s + 1) & 1), Tb((s + 1) & 1), Rd, split, pp,
                              s + 1 >= 2 && s + 1 < split ? hand(smem, s + 1) : nullptr);
            } else {
                for (int j = s + 1 + w; j < split; j += NWAVES - 1) {
                    Strip<B> C;
                    strip_load<B>(C, Aik + (size_t)16 * j * B, B);
                    panel_update<B, 16, true, true>(C, Akk + (size_t)16 * j * B, Vs, LDV, Ts, 16 * s);
                    // the next panel but one goes to the handoff buffer (its
                    // panel rewrites the whole strip in memory)
                    if (j == s + 2)
                        strip_to_hand(C, hand(smem, j));
                    else
                        strip_store<B>(C, Aik + (size_t)16 * j * B, B);
                }
            }
            if (pp.prev && t0) pipe_wait_rows(pp, min(s + 2, NB), NB);
            if (pp.mine) release_before_publish();
            __syncthreads();
            // this task's part of row block s is final (the helper's part is
            // published by the helper)
            if (pp.mine && t0) pipe_publish(pp, s + 2 == NB ? NB : s + 1);
        }
    }

    // The helper of TSQRT(i,k): claims strips [help_split(), NB) of A_ik and
    // applies every inner block to them as the TSQRT publishes its panels
    // (pv), publishing the blocks applied (hb); the TSQRT applies the last
    // block to each of those strips itself (the lookahead before its panel).
    // The same operations in the same order on every column as without it.
    __device__ __forceinline__ static void tsqrt16_helper(double *Akk, double *Aik, const double *Tik, double *smem,
                                                          const Pipe &pp) {
        __shared__ int32_t s_ok;
        const bool t0 = threadIdx.x == 0;
        const int w = __builtin_amdgcn_readfirstlane(wave_id());
        if (t0) {
            int32_t expect = 0;
            s_ok = __hip_atomic_compare_exchange_strong(pp.claim, &expect, 2, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                        TQR_FLAG_SCOPE)
                       ? 1
                       : 0;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) return;
        const int split = help_split();
        double *Vl = smem, *Tl = smem + (size_t)LDV * IB;
#pragma unroll 1
        for (int s = 0; s + 2 < NB; ++s) {
            if (t0) {
                // block s rewrites row block s of R_kk over the helper's
                // strips: the predecessor (and its helper) must be done with
                // it, and this task's panel s must be stored
                if (pp.prev) pipe_wait_rows(pp, s + 1, NB);
                pipe_wait_on(pp, pp.pv, s + 1);
            }
            __syncthreads();
            stage(Aik, Tik, 16 * s, Vl, Tl);
            __syncthreads();
            for (int j = max(split, s + 2) + w; j < NB; j += NWAVES) {
                Strip<B> C;
                strip_load<B>(C, Aik + (size_t)16 * j * B, B);
                panel_update<B, 16, true, true>(C, Akk + (size_t)16 * j * B, Vl, LDV, Tl, 16 * s);
                strip_store<B>(C, Aik + (size_t)16 * j * B, B);
            }
            release_before_publish();
            __syncthreads();
            if (t0) pipe_publish_on(pp.hb, s + 1);
        }
    }

    __device__ __forceinline__ static void tsqrt16_panel(double *Akk, double *Aik, double *Tik, int j, const double *Vs,
                                                         const double *Ts, double *Vn, double *Tn, double *Rd, int split,
                                                         const Pipe &pp, const double *H) {
        const int l = lane_id();
        const int cj = 16 * j;
        double *acol = Aik + (size_t)cj * B, *rcol = Akk + (size_t)cj * B;
        // the diagonal block of R (upper triangle), row-major with row r
        // rotated left by panel_rot(r) (the layout ts_panel16u works in); the
        // lookahead does not touch it, so its load is issued first
        double rdv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = l + 64 * q, r = idx >> 4, c = (panel_rot<PU>(r) + (idx & 15)) & 15;
            rdv[q] = r <= c ? rcol[(size_t)c * B + cj + r] : 0.0;
        }
        // a helper strip has blocks 0 .. j-2 applied by the helper
        if (j >= split && threadIdx.x == 0) pipe_wait_on(pp, pp.hb, j - 1);
        {
            Strip<B> C;
            // the strip comes from the handoff buffer when one is given
            if (H)
                hand_to_strip(C, H);
            else
                strip_load<B>(C, acol, B);
            if (j > 0) panel_update<B, 16, true, true>(C, rcol, Vs, LDV, Ts, cj - 16);
            strip_to_lds(C, Vn);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Rd[l + 64 * q] = rdv[q];
        double x[RPL][16];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = l + 64 * i;
#pragma unroll
            for (int c = 0; c < 16; ++c) x[i][c] = r < B ? Vn[c * LDV + r] : 0.0;
        }
        ts_panel16u<RPL, PU>(x, Rd, Tn, Rd + 256);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = l + 64 * i;
            if (r < B) {
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    acol[(size_t)c * B + r] = x[i][c];
                    Vn[c * LDV + r] = x[i][c];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = l + 64 * q, r = idx >> 4, c = (panel_rot<PU>(r) + (idx & 15)) & 15;
            if (r <= c) rcol[(size_t)c * B + cj + r] = Rd[idx];
            Tik[(size_t)cj * 16 + idx] = Tn[idx];
        }
        // V and T of panel j are stored: for the helper and the SSRFB that
        // follow this task
        if (pp.pv && threadIdx.x == 0) pipe_publish_on(pp.pv, j + 1);
    }

    struct Lds {
        double *P, *Ts, *G, *tau, *wv, *red;
        __device__ explicit Lds(double *base) {
            P = base;
            Ts = P + PANEL_DOUBLES;
            G = Ts + IB * IB;
            tau = G + IB * IB;
            wv = tau + IB;
            red = wv + IB;
        }
    };

    // DGEQT2 (GEQRT): A_kk <- V_kk, R_kk; T_kk written; Vkk receives V_kk as
    // a dense unit-lower matrix for the LARFB tasks.
    __device__ __forceinline__ static void geqrt(double *Akk, double *Tkk, double *Vkk, double *smem, const Pipe &pp) {
        if constexpr (IB == 16) {
            geqrt16(Akk, Tkk, Vkk, smem, pp);
            return;
        }
        Lds L(smem);
        const int tid = threadIdx.x;
#pragma unroll 1
        for (int s = 0; s < NB; ++s) {
            const int c0 = s * IB, hp = B - c0;
            for (int idx = tid; idx < hp * IB; idx += NT) {
                const int r = idx % hp, c = idx / hp;
                L.P[(size_t)c * LDP + r] = Akk[(size_t)(c0 + c) * B + c0 + r];
            }
            __syncthreads();
            panel_factor<IB>(L.P, hp, LDP, L.tau, L.wv, L.red);
            panel_t<IB>(L.P, hp, LDP, L.tau, L.Ts, L.G);
            for (int idx = tid; idx < hp * IB; idx += NT) {
                const int r = idx % hp, c = idx / hp;
                Akk[(size_t)(c0 + c) * B + c0 + r] = L.P[(size_t)c * LDP + r];
            }
            for (int idx = tid; idx < B * IB; idx += NT) {
                const int r = idx % B, c = idx / B;
                const double x = r < c0 + c ? 0.0 : (r == c0 + c ? 1.0 : L.P[(size_t)c * LDP + r - c0]);
                Vkk[(size_t)(c0 + c) * B + r] = x;
            }
            for (int idx = tid; idx < IB * IB; idx += NT) Tkk[(size_t)c0 * IB + idx] = L.Ts[idx];
            __syncthreads();
            // the panel in LDS becomes the dense unit-lower V of this block
            for (int idx = tid; idx < IB * IB; idx += NT) {
                const int r = idx % IB, c = idx / IB;
                if (r <= c) L.P[(size_t)c * LDP + r] = (r == c) ? 1.0 : 0.0;
            }
            __syncthreads();
            // trailing columns c0+IB..B-1: I - V T^T V^T (V row r of the tile at P row r - c0)
            for (int col0 = c0 + IB + 16 * wave_id(); col0 < B; col0 += WCOLS) {
                Strip<B> C;
                strip_load<B>(C, Akk + (size_t)col0 * B, B);
                panel_update<B, IB, true, false>(C, nullptr, L.P - c0, LDP, L.Ts, c0);
                strip_store<B>(C, Akk + (size_t)col0 * B, B, c0 / 16);
            }
            __syncthreads();
        }
    }

    // DTSQT2 (TSQRT): [R_kk; A_ik] <- R~_kk, V_ik; T_ik written.  Only the
    // upper triangle of the diagonal tile is read or written.
    __device__ __forceinline__ static void tsqrt(double *Akk, double *Aik, double *Tik, double *smem, const Pipe &pp) {
        if constexpr (IB == 16) {
            tsqrt16(Akk, Aik, Tik, smem, pp);
            return;
        }
        Lds L(smem);
        const int tid = threadIdx.x;
        constexpr int hp = IB + B;
#pragma unroll 1
        for (int s = 0; s < NB; ++s) {
            const int c0 = s * IB;
            for (int idx = tid; idx < IB * IB; idx += NT) {
                const int r = idx % IB, c = idx / IB;
                L.P[(size_t)c * LDP + r] = (r <= c) ? Akk[(size_t)(c0 + c) * B + c0 + r] : 0.0;
            }
            for (int idx = tid; idx < B * IB; idx += NT) {
                const int r = idx % B, c = idx / B;
                L.P[(size_t)c * LDP + IB + r] = Aik[(size_t)(c0 + c) * B + r];
            }
            __syncthreads();
            panel_factor<IB>(L.P, hp, LDP, L.tau, L.wv, L.red);
            panel_t<IB>(L.P, hp, LDP, L.tau, L.Ts, L.G);
            for (int idx = tid; idx < IB * IB; idx += NT) {
                const int r = idx % IB, c = idx / IB;
                if (r <= c) Akk[(size_t)(c0 + c) * B + c0 + r] = L.P[(size_t)c * LDP + r];
                Tik[(size_t)c0 * IB + idx] = L.Ts[idx];
            }
            for (int idx = tid; idx < B * IB; idx += NT) {
                const int r = idx % B, c = idx / B;
                Aik[(size_t)(c0 + c) * B + r] = L.P[(size_t)c * LDP + IB + r];
            }
            __syncthreads();
            // trailing columns: V_ik of this block is rows IB.. of the panel in LDS
            for (int col0 = c0 + IB + 16 * wave_id(); col0 < B; col0 += WCOLS) {
                Strip<B> C;
                strip_load<B>(C, Aik + (size_t)col0 * B, B);
                panel_update<B, IB, true, true>(C, Akk + (size_t)col0 * B, L.P + IB, LDP, L.Ts, c0);
                strip_store<B>(C, Aik + (size_t)col0 * B, B);
            }
            __syncthreads();
        }
    }

    // Stage block c0 of a reflector tile (B x IB, column-major, ld B) and its T
    // (IB x IB) in LDS.
    __device__ __forceinline__ static void stage(const double *V, const double *T, int c0, double *Vl, double *Tl) {
        const int tid = threadIdx.x;
        for (int idx = tid; idx < B * IB; idx += NT) {
            const int r = idx % B, c = idx / B;
            Vl[c * LDV + r] = V[(size_t)(c0 + c) * B + r];
        }
        for (int idx = tid; idx < IB * IB; idx += NT) Tl[idx] = T[(size_t)c0 * IB + idx];
    }

    // Register half of the double-buffered staging: this thread's share of
    // block c0 of V (B x IB) and of its T (IB x IB).
    struct StageRegs {
        double v[STAGE_V], t[STAGE_T];
    };
    __device__ __forceinline__ static void stage_fetch(const double *V, const double *T, int c0, StageRegs &R) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int k = 0; k < STAGE_V; ++k) {
            const int idx = tid + k * NT, r = idx % B, c = idx / B;
            R.v[k] = V[(size_t)(c0 + c) * B + r];
        }
#pragma unroll
        for (int k = 0; k < STAGE_T; ++k) {
            const int idx = tid + k * NT;
            R.t[k] = idx < IB * IB ? T[(size_t)c0 * IB + idx] : 0.0;
        }
    }
    // Part k (k = 0 .. B/16-1) of stage_fetch: a 16th-of-the-tile share of
    // V's doubles, and T with part 0; the parts together fetch what
    // stage_fetch does.
    __device__ __forceinline__ static void stage_fetch_part(const double *V, const double *T, int c0, StageRegs &R,
                                                            int k) {
        static_assert(STAGE_V % (B / 16) == 0 || B / 16 % STAGE_V == 0, "stage parts");
        constexpr int PER = STAGE_V >= B / 16 ? STAGE_V / (B / 16) : 1;
        const int tid = threadIdx.x;
        if (STAGE_V >= B / 16 || k < STAGE_V) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int kk = k * PER + u;
                const int idx = tid + kk * NT, r = idx % B, c = idx / B;
                R.v[kk] = V[(size_t)(c0 + c) * B + r];
            }
        }
        if (k == 0) {
#pragma unroll
            for (int u = 0; u < STAGE_T; ++u) {
                const int idx = tid + u * NT;
                R.t[u] = idx < IB * IB ? T[(size_t)c0 * IB + idx] : 0.0;
            }
        }
    }
    __device__ __forceinline__ static void stage_commit(const StageRegs &R, double *buf) {
        const int tid = threadIdx.x;
        double *Vl = buf, *Tl = buf + (size_t)LDV * IB;
#pragma unroll
        for (int k = 0; k < STAGE_V; ++k) {
            const int idx = tid + k * NT, r = idx % B, c = idx / B;
            Vl[c * LDV + r] = R.v[k];
        }
#pragma unroll
        for (int k = 0; k < STAGE_T; ++k) {
            const int idx = tid + k * NT;
            if (idx < IB * IB) Tl[idx] = R.t[k];
        }
    }

    // LARFB / SSRFB with double-buffered staging: block si+1 is fetched into
    // registers before block si is applied and written to the other buffer
    // after, so its load latency overlaps the matrix-core work; one barrier
    // per block.  For SSRFB the wave's top rows of the block are loaded first,
    // so that waiting for them does not wait for the prefetch.
    template <bool TRANS, bool TS>
    // With pp.prev (forward order only) the reflectors are those of a TSQRT
    // still running: block s is read once that task has stored panel s
    // (its panel word pp.prev reaches s + 1).
    __device__ __forceinline__ static void apply_dbuf(Strip<B> &C, double *Top, const double *V, const double *T,
                                                      int col0, bool owner, double *smem, const Pipe &pp = Pipe{}) {
        auto buf = [smem](int x) { return smem + (x & 1) * STAGE_DOUBLES; };
        const bool t0 = threadIdx.x == 0;
        StageRegs R;
        if (TRANS && pp.prev) {
            if (t0) pipe_wait(pp, min(2, NB));  // blocks 0 and 1
            __syncthreads();
        }
        stage_fetch(V, T, (TRANS ? 0 : NB - 1) * IB, R);
        stage_commit(R, buf(0));
        __syncthreads();
#pragma unroll 1
        for (int si = 0; si < NB; ++si) {
            const int c0 = (TRANS ? si : NB - 1 - si) * IB;
            double *cur = buf(si & 1);
            d4 Wt[IB / 16];
            if (TS) load_top<B, IB>(Wt, Top + (size_t)col0 * B, c0);
            // the prefetch of block si+1, one part per row block of the
            // products (after the last block a block is fetched again and
            // dropped, which keeps the issue free of branches)
            const int cn = (TRANS ? min(si + 1, NB - 1) : max(NB - 2 - si, 0)) * IB;
            auto issue = [&](int k) { stage_fetch_part(V, T, cn, R, k); };
            panel_update<B, IB, TRANS, TS>(C, TS ? Top + (size_t)col0 * B : nullptr, cur, LDV, cur + (size_t)LDV * IB,
                                           c0, owner, TS ? Wt : nullptr, issue);
            if (si + 1 < NB) stage_commit(R, buf((si + 1) & 1));
            if (TRANS && pp.prev && t0 && si + 2 < NB) pipe_wait(pp, si + 3);  // block si+2, fetched next
            __syncthreads();
        }
    }

    // DLARFB (LARFB) on columns [cbeg, cend) of a b-row tile with the
    // reflectors of a diagonal tile (Vd: V_kk as a dense unit-lower matrix,
    // T_kk): C <- Q_kk^T C (trans) or Q_kk C.  With pp.prev (forward order
    // only) the reflectors are those of a GEQRT still running, followed
    // block by block as apply_dbuf does.
    template <bool TRANS>
    __device__ __forceinline__ static void larfb(const double *Vd, const double *Tkk, double *Cb, int cbeg, int cend,
                                                 double *smem, const Pipe &pp = Pipe{}) {
        double *Vl = smem, *Tl = smem + (size_t)LDV * IB;
        // every wave works on a valid strip (waves past the end repeat the last
        // one) so that the strip's registers have a single definition; only
        // the owning wave stores
        const int want = cbeg + 16 * wave_id();
        const int col0 = min(want, cend - 16);
        const bool owner = want < cend;
        Strip<B> C;
        strip_load<B>(C, Cb + (size_t)col0 * B, B);
        if constexpr (DBUF) {
            apply_dbuf<TRANS, false>(C, nullptr, Vd, Tkk, col0, owner, smem, pp);
        } else {
#pragma unroll 1
            for (int si = 0; si < NB; ++si) {
                const int c0 = (TRANS ? si : NB - 1 - si) * IB;
                __syncthreads();
                stage(Vd, Tkk, c0, Vl, Tl);
                __syncthreads();
                panel_update<B, IB, TRANS, false>(C, nullptr, Vl, LDV, Tl, c0);
            }
        }
        if (owner) strip_store<B>(C, Cb + (size_t)col0 * B, B);
    }

    // DSSRFB (SSRFB) on columns [cbeg, cend) of the pair (top, C) with the
    // reflectors (V_ik, T_ik) of a TSQRT tile.
    template <bool TRANS>
    __device__ __forceinline__ static void ssrfb(double *Top, double *Cb, const double *Vik, const double *Tik, int cbeg, int cend,
                                 double *smem, const Pipe &pp = Pipe{}) {
        double *Vl = smem, *Tl = smem + (size_t)LDV * IB;
        const int want = cbeg + 16 * wave_id();
        const int col0 = min(want, cend - 16);
        const bool owner = want < cend;
        Strip<B> C;
        strip_load<B>(C, Cb + (size_t)col0 * B, B);
        if constexpr (DBUF) {
            apply_dbuf<TRANS, true>(C, Top, Vik, Tik, col0, owner, smem, pp);
        } else {
#pragma unroll 1
            for (int si = 0; si < NB; ++si) {
                const int c0 = (TRANS ? si : NB - 1 - si) * IB;
                __syncthreads();
                stage(Vik, Tik, c0, Vl, Tl);
                __syncthreads();
                panel_update<B, IB, TRANS, true>(C, Top + (size_t)col0 * B, Vl, LDV, Tl, c0, owner);
            }
        }
        if (owner) strip_store<B>(C, Cb + (size_t)col0 * B, B);
    }

    // ---- FP32 precision tier of LARFB / SSRFB (inner block 16) -----------
    // V and T of a block are fetched as FP64 and written to LDS as floats;
    // the strip is converted to float once when loaded and back when stored.
    __device__ __forceinline__ static void stage_commit_f(const StageRegs &R, float *buf) {
        const int tid = threadIdx.x;
        float *Vl = buf, *Tl = buf + (size_t)LDV * IB;
#pragma unroll
        for (int k = 0; k < STAGE_V; ++k) {
            const int idx = tid + k * NT, r = idx % B, c = idx / B;
            Vl[c * LDV + r] = (float)R.v[k];
        }
#pragma unroll
        for (int k = 0; k < STAGE_T; ++k) {
            const int idx = tid + k * NT;
            if (idx < IB * IB) Tl[idx] = (float)R.t[k];
        }
    }

    template <bool TRANS, bool TS, bool BF16 = false>
    __device__ __forceinline__ static void apply_dbuf_f32(StripF<B> &C, double *Top, const double *V, const double *T,
                                                          int col0, bool owner, double *smem, const Pipe &pp = Pipe{}) {
        static_assert(IB == 16, "the FP32 tier works with inner block 16");
        constexpr size_t STAGE_F = (size_t)LDV * IB + IB * IB;
        float *fb = reinterpret_cast<float *>(smem);
        auto buf = [fb](int x) { return fb + (x & 1) * STAGE_F; };
        const bool t0 = threadIdx.x == 0;
        StageRegs R;
        if (TRANS && pp.prev) {
            if (t0) pipe_wait(pp, min(2, NB));
            __syncthreads();
        }
        stage_fetch(V, T, (TRANS ? 0 : NB - 1) * IB, R);
        stage_commit_f(R, buf(0));
        __syncthreads();
#pragma unroll 1
        for (int si = 0; si < NB; ++si) {
            const int c0 = (TRANS ? si : NB - 1 - si) * IB;
            float *cur = buf(si & 1);
            if (si + 1 < NB) stage_fetch(V, T, (TRANS ? si + 1 : NB - 2 - si) * IB, R);
            panel_update_f32<B, TRANS, TS, BF16>(C, TS ? Top + (size_t)col0 * B : nullptr, cur, LDV,
                                                 cur + (size_t)LDV * IB, c0, owner);
            if (si + 1 < NB) stage_commit_f(R, buf((si + 1) & 1));
            if (TRANS && pp.prev && t0 && si + 2 < NB) pipe_wait(pp, si + 3);
            __syncthreads();
        }
    }

    template <bool TRANS, bool BF16 = false>
    __device__ __forceinline__ static void larfb_f32(const double *Vd, const double *Tkk, double *Cb, int cbeg, int cend,
                                                     double *smem, const Pipe &pp = Pipe{}) {
        const int want = cbeg + 16 * wave_id();
        const int col0 = min(want, cend - 16);
        const bool owner = want < cend;
        StripF<B> C;
        strip_load_f<B>(C, Cb + (size_t)col0 * B, B);
        apply_dbuf_f32<TRANS, false, BF16>(C, nullptr, Vd, Tkk, col0, owner, smem, pp);
        if (owner) strip_store_f<B>(C, Cb + (size_t)col0 * B, B);
    }

    template <bool TRANS, bool BF16 = false>
    __device__ __forceinline__ static void ssrfb_f32(double *Top, double *Cb, const double *Vik, const double *Tik, int cbeg,
                                                     int cend, double *smem, const Pipe &pp = Pipe{}) {
        const int want = cbeg + 16 * wave_id();
        const int col0 = min(want, cend - 16);
        const bool owner = want < cend;
        StripF<B> C;
        strip_load_f<B>(C, Cb + (size_t)col0 * B, B);
        apply_dbuf_f32<TRANS, true, BF16>(C, Top, Vik, Tik, col0, owner, smem, pp);
        if (owner) strip_store_f<B>(C, Cb + (size_t)col0 * B, B);
    }
};

// ---------------------------------------------------------------------------
// Task bodies
// ---------------------------------------------------------------------------
// F32: LARFB/SSRFB on the FP32 matrix cores; with BF as well, their two
// large products take BF16 operands (FP32 accumulation).
template <int B, int IB, bool F32 = false, bool BF = false>
struct FactorBody {
    using K = TileKernels<B, IB>;
    double *W;   // tiles
    double *T;   // T slots
    double *Vd;  // dense unit-lower V of each diagonal tile
    int p;
    // pipelined R_kk chain (inner block 16, persistent mode): progress word
    // of chain task (i,k) at prog[k*p + i]; null runs every chain task only
    // after its predecessor has finished
    int32_t *prog = nullptr;
    int32_t *status = nullptr;
    int64_t wait_ticks = 0;
    int q = 0;             // tile columns (the progress words are four p x q arrays)
    bool helpers = false;  // TSQRT tasks have helper tasks in the graph
    __device__ double *tile(int i, int j) const { return W + ((int64_t)j * p + i) * B * B; }
    __device__ Pipe pipe(const Task &t) const {
        Pipe pp{nullptr, nullptr, status, 0};
        if (prog) {
            // words of chain task (i,k): R_kk row blocks finished, panels
            // stored, blocks applied by the helper, claim of the helper strips
            const int64_t pq = (int64_t)p * q, row = (int64_t)t.k * p;
            int32_t *panels = prog + pq + row, *helped = prog + 2 * pq + row, *claim = prog + 3 * pq + row;
            if (t.kind == TSQRT || t.kind == TSQRT_HELP) {
                pp.prev = prog + row + t.i - 1;  // the predecessor on the R_kk chain
                pp.mine = t.kind == TSQRT ? prog + row + t.i : nullptr;  // read by TSQRT(i+1,k)
                pp.pv = panels + t.i;
                pp.hb = helped + t.i;
                if (helpers) pp.claim = claim + t.i;
                if (helpers && t.i - 1 > t.k) {
                    pp.prev_hb = helped + t.i - 1;
                    pp.prev_claim = claim + t.i - 1;
                }
            } else if (t.kind == GEQRT) {
                pp.mine = prog + row + t.i;  // read by TSQRT(k+1,k) and LARFB(k,k+1,c)
            } else if (t.kind == LARFB && t.j == t.k + 1) {
                pp.prev = prog + row + t.k;  // the V and T panels GEQRT(k) has stored
            } else if (t.kind == SSRFB && t.j == t.k + 1) {
                pp.prev = panels + t.i;  // the panels of the TSQRT(i,k) whose reflectors it applies
            }
            pp.deadline = rt_clock() + (uint64_t)wait_ticks;
        }
        return pp;
    }
    __device__ double *tslot(int i, int k) const { return T + ((int64_t)k * p + i) * IB * B; }
    __device__ double *vdiag(int k) const { return Vd + (int64_t)k * B * B; }
    __device__ __forceinline__ void run(const Task &t, double *smem) const {
        const int cbeg = t.c * kStripCols, cend = min(B, cbeg + kStripCols);
        switch (t.kind) {
        case GEQRT: K::geqrt(tile(t.k, t.k), tslot(t.k, t.k), vdiag(t.k), smem, pipe(t)); break;
        case TSQRT: K::tsqrt(tile(t.k, t.k), tile(t.i, t.k), tslot(t.i, t.k), smem, pipe(t)); break;
        case TSQRT_HELP:
            if constexpr (IB == 16) K::tsqrt16_helper(tile(t.k, t.k), tile(t.i, t.k), tslot(t.i, t.k), smem, pipe(t));
            break;
        case LARFB:
            if constexpr (F32)
                K::template larfb_f32<true, BF>(vdiag(t.k), tslot(t.k, t.k), tile(t.k, t.j), cbeg, cend, smem, pipe(t));
            else
                K::template larfb<true>(vdiag(t.k), tslot(t.k, t.k), tile(t.k, t.j), cbeg, cend, smem, pipe(t));
            break;
        default:
            if constexpr (F32)
                K::template ssrfb_f32<true, BF>(tile(t.k, t.j), tile(t.i, t.j), tile(t.i, t.k), tslot(t.i, t.k), cbeg,
                                                cend, smem, pipe(t));
            else
                K::template ssrfb<true>(tile(t.k, t.j), tile(t.i, t.j), tile(t.i, t.k), tslot(t.i, t.k), cbeg, cend, smem,
                                        pipe(t));
            break;
        }
    }
};

// Q^T (TRANS) or Q applied to the p row tiles of B (b x wb each).
template <int B, int IB, bool TRANS>
struct ApplyBody {
    using K = TileKernels<B, IB>;
    const double *W;
    const double *T;
    const double *Vd;  // dense unit-lower V of each diagonal tile
    double *Bt;
    int p, wb;
    __device__ const double *tile(int i, int j) const { return W + ((int64_t)j * p + i) * B * B; }
    __device__ const double *tslot(int i, int k) const { return T + ((int64_t)k * p + i) * IB * B; }
    __device__ double *btile(int i) const { return Bt + (int64_t)i * B * wb; }
    __device__ __forceinline__ void run(const Task &t, double *smem) const {
        const int cbeg = t.c * kStripCols, cend = min(wb, cbeg + kStripCols);
        if (t.i == t.k)
            K::template larfb<TRANS>(Vd + (int64_t)t.k * B * B, tslot(t.k, t.k), btile(t.k), cbeg, cend, smem);
        else
            K::template ssrfb<TRANS>(btile(t.k), btile(t.i), tile(t.i, t.k), tslot(t.i, t.k), cbeg, cend, smem);
    }
};

// Back substitution X = R^{-1} Y with the upper tiles of R; Y/X in the row
// tiles of B (b x wb).  nrow = n (rows of R that are not padding).
template <int B>
struct TrsmBody {
    const double *W;
    double *Bt;
    int p, wb;
    int64_t nrow;
    __device__ const double *tile(int i, int j) const { return W + ((int64_t)j * p + i) * B * B; }
    __device__ double *btile(int i) const { return Bt + (int64_t)i * B * wb; }
    __device__ __forceinline__ void run(const Task &t, double *smem) const {
        if (t.kind == 1) {
            // G(i,j): B_i -= R_ij X_j on the matrix cores
            const double *R = tile(t.i, t.j);
            const double *X = btile(t.j);
            double *Y = btile(t.i);
            const int l = lane_id();
            for (int col0 = 16 * wave_id(); col0 < wb; col0 += 16 * NWAVES) {
                Strip<B> C;
                strip_load<B>(C, Y + (size_t)col0 * B, B);
                // k-slice (kb, r): rows 16kb + 4r .. +3 of X_j, columns of R
                const double *xp = X + (size_t)(col0 + (l & 15)) * B + (l >> 4);
                const double *rp = R + (size_t)(l >> 4) * B + strip_row_perm(l & 15);
#pragma unroll 1
                for (int kb = 0; kb < B / 16; ++kb) {
                    const d4 x = -ld4s(xp + 16 * kb, 4);
                    const double *rk = rp + (size_t)16 * kb * B;
#pragma unroll
                    for (int rb = 0; rb < B / 16; ++rb) {
                        const double *q = rk + 16 * rb;
                        C.v[rb] = mfma(q[0], x.x, C.v[rb]);
                        C.v[rb] = mfma(q[4 * B], x.y, C.v[rb]);
                        C.v[rb] = mfma(q[8 * B], x.z, C.v[rb]);
                        C.v[rb] = mfma(q[12 * B], x.w, C.v[rb]);
                    }
                }
                strip_store<B>(C, Y + (size_t)col0 * B, B);
            }
            return;
        }
        // D(i): solve R_ii X_i = Y_i for the rows that are not padding;
        // padding rows of X_i are set to zero.
        const double *R = tile(t.i, t.i);
        double *Y = btile(t.i);
        const int64_t rem = nrow - (int64_t)t.i * B;
        const int nloc = (int)(rem < B ? rem : B);
        const int tid = threadIdx.x;
        double *y = smem;  // B x 16
        for (int g0 = 0; g0 < wb; g0 += 16) {
            for (int idx = tid; idx < B * 16; idx += NT) {
                const int r = idx % B, c = idx / B;
                y[idx] = (r < nloc) ? Y[(size_t)(g0 + c) * B + r] : 0.0;
            }
            __syncthreads();
            for (int cidx = nloc - 1; cidx >= 0; --cidx) {
                const double *rc = R + (size_t)cidx * B;
                if (tid < 16) y[cidx + tid * B] = y[cidx + tid * B] / rc[cidx];
                __syncthreads();
                for (int idx = tid; idx < cidx * 16; idx += NT) {
                    const int r = idx % cidx, c = idx / cidx;
                    y[r + c * B] -= rc[r] * y[cidx + c * B];
                }
                __syncthreads();
            }
            for (int idx = tid; idx < B * 16; idx += NT) {
                const int r = idx % B, c = idx / B;
                Y[(size_t)(g0 + c) * B + r] = y[idx];
            }
            __syncthreads();
        }
    }
};

// ===========================================================================
// The persistent scheduler: every workgroup repeatedly takes the
// highest-priority ready task, runs it, and releases its successors; a
// successor whose last dependency is released is pushed on its level's queue.
// ===========================================================================
// Successors a task releases when it starts rather than when it ends (they
// follow its progress word inside their bodies): with the pipelined chain,
// TSQRT(i+1,k) after GEQRT(k) (i = k) or TSQRT(i,k), the strips of
// LARFB(k,k+1) after GEQRT(k), and the strips of SSRFB(i,k+1,k) after
// TSQRT(i,k).  They are the first successors in the graph's order; returns
// how many.
// Early successors of one task, at most: a helper, the chain successor and
// one per strip (at most 4 strips per tile).
constexpr int kMaxEarly = 6;
template <class G, class Body>
__device__ __forceinline__ int early_successors(const G &, const Body &, const Task &) { return 0; }
template <int B, int IB, bool F32, bool BF>
__device__ __forceinline__ int early_successors(const FactorGraph &g, const FactorBody<B, IB, F32, BF> &b, const Task &t) {
    static_assert((B > kStripCols ? B / kStripCols : 1) + 2 <= kMaxEarly, "more early successors than kMaxEarly");
    if (!b.prog || (t.kind != GEQRT && t.kind != TSQRT)) return 0;
    const int chain = t.i + 1 < g.p ? 1 : 0;
    if (t.kind == GEQRT) return chain + (t.k + 1 < g.q ? (int)g.S : 0);
    if (t.kind != TSQRT) return 0;
    return (g.helpers ? 1 : 0) + chain + (t.k + 1 < g.q ? (int)g.S : 0);
}

constexpr int kReadyCap = 64;  // ready successors collected per task before publishing
constexpr int kEarlyThread = 128;  // thread 0 of wavefront 2 releases the early successors
static_assert(kEarlyThread < NT, "the releasing thread must exist");

template <class G, class Body>
__global__ void __launch_bounds__(NT) k_persistent(G g, Body body, Sched s, RunOpts o) {
    extern __shared__ double smem[];
    __shared__ int32_t s_task, s_cont, s_nready, s_nover, s_panel;
    __shared__ int32_t s_ready[kReadyCap];
    __shared__ int8_t s_lvl[kReadyCap];
    const int tid = threadIdx.x;
    const int nworkers = gridDim.x;
    // Thread 0 owns the scheduling decisions: the next task is either the
    // continuation chosen at the end of the previous task or one taken from
    // the ready queues.  The task id is made wave-uniform with readfirstlane,
    // so the loop exit is a scalar branch and every lane of every wave meets
    // each barrier in the same iteration.
    uint32_t nsinks = 0;
    if (tid == 0) nsinks = flag_load(&s.st->nsinks);
    int32_t next = -1;  // thread 0: continuation task or -1
    for (;;) {
        if (tid == 0) {
            s_cont = next >= 0;
            s_task = next >= 0 ? next
                               : idle_wait(g, o.policy, o.far_every, s, nsinks, o.abort_flag,
                                           rt_clock() + (uint64_t)o.timeout,
                                           blockIdx.x, nworkers);
            s_nready = 0;
            s_nover = 0;
        }
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_task);
        if (t < 0) break;
        const int cont = __builtin_amdgcn_readfirstlane(s_cont);
        const uint64_t t_pop = o.trace ? rt_clock() : 0;
        // acquire the predecessors' writes; the barrier orders every wave's
        // loads after it
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const Task task = g.decode(t);
        if constexpr (std::is_same<G, FactorGraph>::value) {
            // GEQRT(k) starts in order of k: k+1 panels have started
            if (task.kind == GEQRT && tid == 0)
                __hip_atomic_store(&s.st->panel, task.k + 1, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
        }
        // Successors that follow this task's progress may start as soon as
        // it has started.  Thread 0 of wavefront 2 releases them while the
        // body begins: the bodies that have such successors (GEQRT, TSQRT)
        // start with wavefront 0 alone on its first panel, so the memory
        // round trips of the release are off their critical path.  The
        // counter decrements are issued together, then the pushes.
        const int nearly = early_successors(g, body, task);
        if (nearly > 0 && tid == kEarlyThread) {
            const int panel = flag_load(&s.st->panel);
            int32_t old[kMaxEarly];
#pragma unroll
            for (int n = 0; n < kMaxEarly; ++n)
                old[n] = n < nearly ? __hip_atomic_fetch_add(&s.cnt[g.successor(task, n)], -1, __ATOMIC_RELAXED,
                                                             TQR_FLAG_SCOPE)
                                    : 0;
            int pushed = 0;
#pragma unroll
            for (int n = 0; n < kMaxEarly; ++n) {
                if (old[n] != 1) continue;
                const int64_t e = g.successor(task, n);
                push_one(s, level_of(g, g.decode(e), o.policy, panel), (int32_t)e);
                ++pushed;
            }
            if (pushed > 0) wake_idle(s, pushed, nworkers);
        }
        const uint64_t t_acq = o.trace ? rt_clock() : 0;
        body.run(task, smem);
        const uint64_t t_body = o.trace ? rt_clock() : 0;
        // thread 0 reads the queue words and the status now: the reads
        // complete during the store wait below
        uint64_t qw[kLevels];
        int32_t stat = 0;
        if (tid == 0) {
            read_queue_words(s, qw);
            stat = flag_load(&s.st->status);
        }
        // release the task's writes before its successors are told: every
        // wave waits for its own stores, then one agent-scope release (an L2
        // writeback) by thread 0 covers all of them
        wait_own_stores();
        if (tid == 0) s_panel = flag_load(&s.st->panel);
        __syncthreads();
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        const int panel = s_panel;
        if (o.trace && tid == 0 && t < o.ntrace) {
            int64_t *tr = o.trace + kTraceFields * (int64_t)t;
            tr[0] = (int64_t)t_pop;
            tr[1] = (int64_t)t_acq;
            tr[2] = (int64_t)t_body;
            tr[3] = (int64_t)rt_clock();
            tr[4] = blockIdx.x;
            tr[5] = xcc_id();
            tr[6] = hw_id();
            tr[7] = cont;
        }
        // Successors: the last predecessor to finish makes a task ready.
        const int ns = g.num_successors(task);
        for (int n = tid + nearly; n < ns; n += NT) {
            const int64_t sidx = g.successor(task, n);
            const int32_t old = __hip_atomic_fetch_add(&s.cnt[sidx], -1, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            if (old == 1) {
                const int lvl = level_of(g, g.decode(sidx), o.policy, panel);
                const int slot = atomicAdd(&s_nready, 1);
                if (slot < kReadyCap) {
                    s_ready[slot] = (int32_t)sidx;
                    s_lvl[slot] = (int8_t)lvl;
                } else {
                    push_one(s, lvl, (int32_t)sidx);
                    atomicAdd(&s_nover, 1);
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            next = -1;
            if (ns == 0) {
                const uint32_t d = __hip_atomic_fetch_add(&s.st->done, 1u, __ATOMIC_RELAXED, TQR_FLAG_SCOPE) + 1;
                if (d == nsinks) broadcast_stop(s, nworkers);
            }
            const int nr = min(s_nready, kReadyCap);
            // keep the highest-priority ready successor (lowest level, then
            // lowest id) unless a queue holds work of a higher priority;
            // publish the rest, one queue-word update per level
            int best = -1, best_lvl = kLevels;
            for (int r = 0; r < nr; ++r) {
                const int lvl = s_lvl[r];
                if (lvl < best_lvl || (lvl == best_lvl && s_ready[r] < s_ready[best])) {
                    best = r;
                    best_lvl = lvl;
                }
            }
            if (best >= 0 && queue_has_level_below(qw, best_lvl)) best = -1;
            // the continuation is not published; the rest go to idle
            // workers first (highest priority first), then to the queues
            if (best >= 0) s_lvl[best] = -1;
            handoff_ready(s, s_ready, s_lvl, nr, nworkers);
            int pushed = s_nover;
            for (int l = 0; l < kLevels; ++l) {
                int c = 0;
                for (int r = 0; r < nr; ++r) c += (r != best && s_lvl[r] == l);
                if (c == 0) continue;
                const uint32_t base = (uint32_t)(
                    __hip_atomic_fetch_add(&s.st->ht[l], (uint64_t)c << 32, __ATOMIC_RELAXED, TQR_FLAG_SCOPE) >> 32);
                int i = 0;
                for (int r = 0; r < nr; ++r)
                    if (r != best && s_lvl[r] == l)
                        __hip_atomic_store(&s.queue[l * s.cap + base + i++], s_ready[r], __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
                pushed += c;
            }
            if (pushed > 0) wake_idle(s, pushed, nworkers);
            if (best >= 0) next = s_ready[best];
            // a failed or aborted run takes no continuation (idle_wait sees
            // the status and ends the worker)
            if (stat != 0) next = -1;
        }
    }
}

// One task per launch (reference order; no scheduler state).
template <class G, class Body>
__global__ void __launch_bounds__(NT) k_one_task(G g, Body body, int64_t t) {
    extern __shared__ double smem[];
    body.run(g.decode(t), smem);
}

// Small kernels (defined in tqr.hip).
__global__ void k_copy_status(const SchedState *st, int32_t *out, int only_errors);
__global__ void k_set_int(int32_t *out, int32_t v);
__global__ void k_fill_int(int32_t *out, int64_t n, int32_t v);
__global__ void k_fill_u64(uint64_t *out, int64_t n, uint64_t v);
__global__ void k_unit_lower(const double *__restrict__ W, int p, int b, double *__restrict__ Vd);
__global__ void k_eye(double *Q, int64_t ldq, int64_t m);
constexpr int kResidChunks = 16;
__global__ void k_resid_partial(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int64_t ldx,
                                int nrhs, double *Part, const int32_t *skip);
__global__ void k_sum_chunks(const double *Part, int chunks, int64_t m, int nrhs, double *Q);
struct CglsState;
__global__ void k_resid_replace(const double *Bm, int64_t ldb, const double *Part, int chunks, int64_t m, int nrhs,
                                double *Rv, const CglsState *st);
__global__ void k_gemv_t(const double *A, int64_t lda, int64_t m, const double *Rv, int nrhs, double *G, int64_t n,
                         const int32_t *skip);
__global__ void k_col_sumsq(const double *A, int64_t lda, int64_t m, double *out);
__global__ void k_sum_vec(const double *v, int64_t n, double *out);
// CGLS state of one right-hand side (device)
struct CglsState {
    double gamma;     // ||s||^2 of the current s = R^{-T} A^T r
    double alpha;     // step of the current iteration
    double beta;      // p = s + beta p
    double eta;       // ||R^{-T} A^T r|| / (||A||_F ||x||) at the last test
    double best;      // smallest ||s||^2 seen
    int32_t active;   // 0 once the column has stopped
    int32_t iters;    // iterations applied
    int32_t stop;     // TQR_REFINE_* reason
    int32_t since;    // tests since the smallest ||s||^2 was last halved
};
__global__ void k_cgls_start(const double *S, int64_t n, double *P, const double *Rv, int64_t m, int nrhs,
                             CglsState *st, int max_iter);
__global__ void k_cgls_step(const double *Q, int64_t m, int nrhs, CglsState *st);
__global__ void k_cgls_update_xr(double *Xv, const double *Tv, int64_t n, double *Rv, const double *Q, int64_t m,
                                 int nrhs, const CglsState *st);
__global__ void k_cgls_next(const double *S, const double *Xv, const double *Rv, int64_t n, int64_t m, int nrhs,
                            const double *fro2, CglsState *st, int iter);
__global__ void k_cgls_update_p(double *P, const double *S, int64_t n, int nrhs, const CglsState *st);
__global__ void k_cgls_report(const CglsState *st, int nrhs, tqr_refine_stats *out);
__global__ void k_cgls_alldone(const CglsState *st, int nrhs, int32_t *done);
__global__ void k_refine_stats_empty(tqr_refine_stats *out, int64_t nrhs);
__global__ void k_copy_cm(const double *S, int64_t lds, double *D, int64_t ldd, int64_t rows, int nrhs, double scale);
__global__ void k_diag_info(const double *W, int p, int b, int64_t n, int32_t *info);

// ===========================================================================
// Host side
// ===========================================================================
// Last error of the calling host thread (defined in tqr.hip).
extern thread_local std::string g_err;

inline tqr_status set_err(tqr_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return ::tqr::set_err(TQR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

inline bool tiles_ok(int b, int ib) {
    const bool bok = b == 16 || b == 32 || b == 64 || b == 128 || b == 256;
    const bool iok = ib == 16 || ib == 32 || ib == 64;
    return bok && iok && ib <= b && b % ib == 0 && ib * (b + ib) <= 9216;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }
inline int64_t wb_of(int64_t nrhs) { return cdiv(std::max<int64_t>(nrhs, 1), 16) * 16; }

#include "tqr_narrow.h"

inline bool narrow_ok(int b, int ib, int64_t nrhs) { return ib == 16 && b >= 64 && nrhs >= 1 && nrhs <= kNarrowRhs; }

// Workspace: [tiles p*q*b*b][dense diagonal V q*b*b][B tiles p*b*wb][scheduler]
// [R_kk chain progress words p*q int32][narrow-rhs words and hand-over blocks]
// The narrow region (only when narrow_ok): 64 control ints (apply: ticket,
// abort at 0, 1; triangular solves: at 2, 3; the refinement's "all columns
// stopped" word at 4), then the apply hand-over blocks (q*p*b*kNarrowRhs
// doubles) and the published solution blocks (one 64 x kNarrowRhs block per
// 64 rows of R).
struct Sizes {
    int64_t p, q, tiles_bytes, vd_bytes, btiles_bytes, sched_bytes, prog_bytes, total;
    int64_t nar_ints, nar_h_bytes, nar_x_bytes, nar_bytes;
    int64_t prog_offset() const { return tiles_bytes + vd_bytes + btiles_bytes + sched_bytes; }
    int64_t narrow_offset() const { return prog_offset() + prog_bytes; }
};

inline Sizes sizes_of(int64_t m, int64_t n, int64_t nrhs, int b) {
    Sizes z;
    z.p = cdiv(std::max<int64_t>(m, 1), b);
    z.q = cdiv(std::max<int64_t>(n, 1), b);
    z.tiles_bytes = align256(z.p * z.q * b * b * 8);
    z.vd_bytes = align256(z.q * b * b * 8);
    z.btiles_bytes = nrhs > 0 ? align256(z.p * b * wb_of(nrhs) * 8) : 0;
    int64_t nt = FactorGraph(z.p, z.q, b, true).num_tasks();
    if (nrhs > 0) {
        nt = std::max(nt, ApplyGraph(z.p, z.q, cdiv(wb_of(nrhs), kStripCols), true).num_tasks());
        nt = std::max(nt, TrsmGraph(z.q).num_tasks());
    }
    z.sched_bytes = align256(sched_bytes(nt));
    z.prog_bytes = align256(4 * z.p * z.q * 4);
    z.nar_ints = z.nar_h_bytes = z.nar_x_bytes = z.nar_bytes = 0;
    if (nrhs >= 1 && nrhs <= kNarrowRhs && b >= 64) {
        const int64_t nb = cdiv(std::max<int64_t>(n, 1), kTrsvRows);
        z.nar_ints = 64;
        z.nar_h_bytes = align256(z.q * z.p * (int64_t)b * kNarrowRhs * 8);
        z.nar_x_bytes = align256(nb * kTrsvRows * kNarrowRhs * 8);
        z.nar_bytes = align256(z.nar_ints * 4) + z.nar_h_bytes + z.nar_x_bytes;
    }
    z.total = z.tiles_bytes + z.vd_bytes + z.btiles_bytes + z.sched_bytes + z.prog_bytes + z.nar_bytes;
    return z;
}

// Pointers into the narrow region of a workspace laid out by sizes_of.
struct NarrowMem {
    int32_t *ints;
    double *H, *X;
    const int32_t *skip = nullptr;  // the triangular solves return at once while *skip != 0
};
inline NarrowMem narrow_mem(void *work, const Sizes &z, int b) {
    (void)b;
    char *base = reinterpret_cast<char *>(work) + z.narrow_offset();
    NarrowMem nm;
    nm.ints = reinterpret_cast<int32_t *>(base);
    nm.H = reinterpret_cast<double *>(base + align256(z.nar_ints * 4));
    nm.X = reinterpret_cast<double *>(base + align256(z.nar_ints * 4) + z.nar_h_bytes);
    return nm;
}

// Two seconds of the device's constant-rate clock: a worker that finds no
// ready task for that long while the graph is unfinished gives up.
inline int64_t default_timeout_ticks() {
    static int64_t ticks = [] {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        return (int64_t)khz * 1000 * 2;
    }();
    return ticks;
}

inline int cu_count() {
    static int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
        return v;
    }();
    return cus;
}

// Algorithm 1 order for the reference (serial) mode (defined in tqr.hip).
std::vector<int64_t> serial_order(const FactorGraph &g);
std::vector<int64_t> serial_order(const ApplyGraph &g);
std::vector<int64_t> serial_order(const TrsmGraph &g);
template <class G>
int64_t trace_count(const G &g) { return g.num_tasks(); }
template <>
inline int64_t trace_count<FactorGraph>(const FactorGraph &g) { return g.num_paper_tasks(); }
// far-first workers: the square or wide factorisation under the column policy
template <class G>
int far_every_of(const G &, int) { return 0; }
template <>
inline int far_every_of<FactorGraph>(const FactorGraph &g, int policy) {
    return policy == TQR_POLICY_COLUMN && g.p <= g.q ? kFarEverySquare : 0;
}

template <class G, class Body>
tqr_status run_graph(const G &g, const Body &body, void *sched_mem, size_t lds, const tqr_options *opt,
                     hipStream_t stream, int32_t *status_out, int status_only_errors = 0) {
    const int64_t nt = g.num_tasks();
    if (nt == 0) return TQR_OK;
    Sched s = sched_at(sched_mem, nt);
    const int mode = opt ? opt->mode : TQR_MODE_PERSISTENT;
    // without options: GEQRT > TSQRT > updates by their column's distance
    // from the current panel (the fastest policy measured)
    const int policy = opt ? opt->policy : TQR_POLICY_COLUMN;
    auto kp = k_persistent<G, Body>;
    auto k1 = k_one_task<G, Body>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr_err == hipSuccess)
            attr_err = hipFuncSetAttribute((const void *)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    HIPCHK(attr_err);
    if (mode == TQR_MODE_SERIAL) {
        if (opt && opt->event_begin) HIPCHK(hipEventRecord((hipEvent_t)opt->event_begin, stream));
        // reference order: task ids of the factorisation graph follow
        // Algorithm 1 step by step; within a step GEQRT, then the LARFB
        // strips, then per row TSQRT and its SSRFB strips.
        for (int64_t t : serial_order(g)) {
            hipLaunchKernelGGL(k1, dim3(1), dim3(NT), lds, stream, g, body, t);
        }
        HIPCHK(hipGetLastError());
        if (opt && opt->event_end) HIPCHK(hipEventRecord((hipEvent_t)opt->event_end, stream));
        if (status_out) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, status_out, 0);
        return TQR_OK;
    }
    const int blocks_init = (int)cdiv(std::max<int64_t>(nt, kMaxWorkers), 256);
    hipLaunchKernelGGL(k_sched_init<G>, dim3(blocks_init), dim3(256), 0, stream, g, s);
    hipLaunchKernelGGL(k_sched_seed<G>, dim3((unsigned)cdiv(nt, 256)), dim3(256), 0, stream, g, s, policy);
    int per_cu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kp, NT, lds));
    int64_t workers = (int64_t)std::max(per_cu, 1) * cu_count();
    if (opt && opt->workgroups > 0) workers = std::min<int64_t>(workers, opt->workgroups);
    workers = std::min<int64_t>(std::min<int64_t>(workers, nt), kMaxWorkers);
    RunOpts ro;
    ro.trace = opt ? opt->trace : nullptr;
    ro.ntrace = trace_count(g);
    ro.abort_flag = opt ? opt->abort_flag : nullptr;
    ro.timeout = (opt && opt->timeout_ticks > 0) ? opt->timeout_ticks : default_timeout_ticks();
    ro.policy = policy;
    ro.far_every = far_every_of(g, policy);
    if (opt && opt->event_begin) HIPCHK(hipEventRecord((hipEvent_t)opt->event_begin, stream));
    hipLaunchKernelGGL(kp, dim3((unsigned)workers), dim3(NT), lds, stream, g, body, s, ro);
    HIPCHK(hipGetLastError());
    if (opt && opt->event_end) HIPCHK(hipEventRecord((hipEvent_t)opt->event_end, stream));
    if (status_out) hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, stream, s.st, status_out, status_only_errors);
    HIPCHK(hipGetLastError());
    return TQR_OK;
}


// The factorisation body; with inner block 16 in persistent mode the R_kk
// chain is pipelined (progress words cleared here, on the stream).
template <int B, int IB, bool F32 = false, bool BF = false>
FactorBody<B, IB, F32, BF> factor_body(double *W, double *T, double *Vd, const Sizes &z, void *work, void *sched,
                                   const tqr_options *opt, hipStream_t stream) {
    FactorBody<B, IB, F32, BF> body{W, T, Vd, (int)z.p};
    const bool serial = opt && opt->mode == TQR_MODE_SERIAL;
    if (IB == 16 && !serial) {
        body.prog = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(work) + z.prog_offset());
        body.status = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(sched) + offsetof(SchedState, status));
        body.wait_ticks = (opt && opt->timeout_ticks > 0) ? opt->timeout_ticks : default_timeout_ticks();
        body.q = (int)z.q;
        // helpers shorten each TSQRT, which paces square problems; on tall
        // ones the chain of TSQRTs down a column paces the run and a helper
        // adds to every link of it
        body.helpers = B >= 128 && z.p <= 2 * z.q;
        const int64_t n = 4 * z.p * z.q;
        hipLaunchKernelGGL(k_fill_int, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, body.prog, n, 0);
    }
    return body;
}

template <int B, int IB>
tqr_status factor_impl(int64_t m, int64_t n, double *A, int64_t lda, double *T, void *work, hipStream_t stream,
                       const tqr_options *opt, bool back_to_cm) {
    const Sizes z = sizes_of(m, n, 0, B);
    double *W = reinterpret_cast<double *>(work);
    double *Vd = reinterpret_cast<double *>(reinterpret_cast<char *>(work) + z.tiles_bytes);
    void *sched = reinterpret_cast<char *>(work) + z.tiles_bytes + z.vd_bytes;
    hipLaunchKernelGGL(k_cm_to_tiles, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, A, lda, m, n, W,
                       (int)z.p, B, B);
    FactorGraph g(z.p, z.q, B);
    tqr_status st;
    if constexpr (IB == 16) {
        if (opt && opt->precision == TQR_PRECISION_FP32_UPDATES) {
            const FactorBody<B, IB, true> body = factor_body<B, IB, true>(W, T, Vd, z, work, sched, opt, stream);
            g.helpers = body.helpers;
            st = run_graph(g, body, sched, TileKernels<B, IB>::LDS_BYTES, opt, stream, opt ? opt->status : nullptr);
        } else if (opt && opt->precision == TQR_PRECISION_BF16_UPDATES) {
            if constexpr (B >= 64) {
                const FactorBody<B, IB, true, true> body =
                    factor_body<B, IB, true, true>(W, T, Vd, z, work, sched, opt, stream);
                g.helpers = body.helpers;
                st = run_graph(g, body, sched, TileKernels<B, IB>::LDS_BYTES, opt, stream, opt ? opt->status : nullptr);
            } else {
                return set_err(-11, "TQR_PRECISION_BF16_UPDATES needs tile_b 64, 128 or 256");
            }
        } else {
            const FactorBody<B, IB> body = factor_body<B, IB>(W, T, Vd, z, work, sched, opt, stream);
            g.helpers = body.helpers;
            st = run_graph(g, body, sched, TileKernels<B, IB>::LDS_BYTES, opt, stream, opt ? opt->status : nullptr);
        }
    } else {
        const FactorBody<B, IB> body = factor_body<B, IB>(W, T, Vd, z, work, sched, opt, stream);
        g.helpers = body.helpers;
        st = run_graph(g, body, sched, TileKernels<B, IB>::LDS_BYTES, opt, stream, opt ? opt->status : nullptr);
    }
    if (st != TQR_OK) return st;
    if (back_to_cm)
        hipLaunchKernelGGL(k_tiles_to_cm, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, W, (int)z.p, B, B,
                           A, lda, m, n);
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

template <int B, int IB>
tqr_status apply_impl(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *T, double *W, const double *Vd,
                      double *Bm, int64_t ldb, double *Bt, void *sched, hipStream_t stream,
                      const tqr_options *opt = nullptr) {
    int32_t *status = opt ? opt->status : nullptr;
    const int64_t p = cdiv(m, B), q = cdiv(n, B), wb = wb_of(nrhs);
    if (Bm)  // else Bt already holds B in tiles
        hipLaunchKernelGGL(k_cm_to_tiles, dim3((unsigned)p, 1), dim3(256), 0, stream, Bm, ldb, m, nrhs, Bt, (int)p, B,
                           (int)wb);
    ApplyGraph g(p, q, cdiv(wb, kStripCols), trans);
    tqr_status st;
    if (trans)
        st = run_graph(g, ApplyBody<B, IB, true>{W, T, Vd, Bt, (int)p, (int)wb}, sched, TileKernels<B, IB>::LDS_BYTES,
                       opt, stream, status, 1);
    else
        st = run_graph(g, ApplyBody<B, IB, false>{W, T, Vd, Bt, (int)p, (int)wb}, sched, TileKernels<B, IB>::LDS_BYTES,
                       opt, stream, status, 1);
    return st;
}

template <int B>
tqr_status trsm_impl(int64_t m, int64_t n, int64_t nrhs, const double *W, double *Bt, void *sched, hipStream_t stream,
                     const tqr_options *opt = nullptr) {
    const int64_t p = cdiv(m, B), q = cdiv(n, B), wb = wb_of(nrhs);
    TrsmGraph g(q);
    return run_graph(g, TrsmBody<B>{W, Bt, (int)p, (int)wb, n}, sched, (size_t)B * 16 * 8, opt, stream,
                     opt ? opt->status : nullptr, 1);
}

// ---- narrow right-hand sides (tqr_narrow.h) --------------------------------
// Q^T B (trans) or Q B in place on the column-major m x nrhs block Bm
// (1 <= nrhs <= kNarrowRhs), one workgroup per row tile.  Control words and
// flags are cleared on the stream first (a fill kernel, no memset).
template <int B, int IB>
tqr_status narrow_apply(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *T, const double *W,
                        const double *Vd, double *Bm, int64_t ldb, const NarrowMem &nm, hipStream_t stream,
                        const tqr_options *opt) {
    if constexpr (IB != 16 || B < 64) {
        return set_err(TQR_EDEVICE, "narrow application needs inner_ib 16 and tile_b >= 64");
    } else {
        const int64_t p = cdiv(m, B), q = cdiv(n, B);
        const int nr = nrhs == 1 ? 1 : (nrhs == 2 ? 2 : 4);
        const int64_t nh = q * p * B * nr;
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, stream, nm.ints, (int64_t)2, 0);
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, stream,
                           reinterpret_cast<uint64_t *>(nm.H), nh, kPendingBits);
        NarrowApplyArgs a;
        a.W = W;
        a.Vd = Vd;
        a.T = T;
        a.Bm = Bm;
        a.ldb = ldb;
        a.m = m;
        a.nrhs = (int)nrhs;
        a.p = (int)p;
        a.q = (int)q;
        a.H = nm.H;
        a.ctl.ticket = nm.ints;
        a.ctl.abort = nm.ints + 1;
        a.ctl.status = opt ? opt->status : nullptr;
        a.ctl.timeout = (opt && opt->timeout_ticks > 0) ? opt->timeout_ticks : default_timeout_ticks();
        const dim3 grid((unsigned)p), block(B);
        if (nrhs == 1) {
            if (trans) hipLaunchKernelGGL((k_narrow_apply<B, IB, 1, true>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((k_narrow_apply<B, IB, 1, false>), grid, block, 0, stream, a);
        } else if (nrhs == 2) {
            if (trans) hipLaunchKernelGGL((k_narrow_apply<B, IB, 2, true>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((k_narrow_apply<B, IB, 2, false>), grid, block, 0, stream, a);
        } else {
            if (trans) hipLaunchKernelGGL((k_narrow_apply<B, IB, 4, true>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((k_narrow_apply<B, IB, 4, false>), grid, block, 0, stream, a);
        }
        HIPCHK(hipGetLastError());
        return TQR_OK;
    }
}

// R X = Y (trans false) or R^T X = Y (trans true) in place on the
// column-major n x nrhs block Y, R the upper triangle of the tiles W.
template <int B>
tqr_status narrow_trsv(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *W, double *Y, int64_t ldy,
                       const NarrowMem &nm, hipStream_t stream, const tqr_options *opt) {
    const int64_t p = cdiv(m, B);
    const int64_t nb = cdiv(n, kTrsvRows);
    const int nr = nrhs == 1 ? 1 : (nrhs == 2 ? 2 : 4);
    const int64_t nx = nb * kTrsvRows * nr;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, stream, nm.ints + 2, (int64_t)2, 0);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)cdiv(nx, 256)), dim3(256), 0, stream,
                       reinterpret_cast<uint64_t *>(nm.X), nx, kPendingBits);
    NarrowTrsvArgs a;
    a.W = W;
    a.p = (int)p;
    a.n = n;
    a.Y = Y;
    a.ldy = ldy;
    a.nrhs = (int)nrhs;
    a.X = nm.X;
    a.skip = nm.skip;
    a.ctl.ticket = nm.ints + 2;
    a.ctl.abort = nm.ints + 3;
    a.ctl.status = opt ? opt->status : nullptr;
    a.ctl.timeout = (opt && opt->timeout_ticks > 0) ? opt->timeout_ticks : default_timeout_ticks();
    const dim3 grid((unsigned)nb), block(256);
    if (nrhs == 1) {
        if (trans) hipLaunchKernelGGL((k_narrow_trsv<B, 1, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_narrow_trsv<B, 1, false>), grid, block, 0, stream, a);
    } else if (nrhs == 2) {
        if (trans) hipLaunchKernelGGL((k_narrow_trsv<B, 2, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_narrow_trsv<B, 2, false>), grid, block, 0, stream, a);
    } else {
        if (trans) hipLaunchKernelGGL((k_narrow_trsv<B, 4, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_narrow_trsv<B, 4, false>), grid, block, 0, stream, a);
    }
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

inline tqr_status check_opts(const tqr_options *o) {
    if (!o) return TQR_OK;
    if (o->struct_size != (int32_t)sizeof(tqr_options)) return -11;
    if (o->mode != TQR_MODE_PERSISTENT && o->mode != TQR_MODE_SERIAL) return -11;
    if (o->policy != TQR_POLICY_PAPER && o->policy != TQR_POLICY_LOOKAHEAD && o->policy != TQR_POLICY_COLUMN)
        return -11;
    if (o->workgroups < 0) return -11;
    if (o->precision != TQR_PRECISION_FP64 && o->precision != TQR_PRECISION_FP32_UPDATES &&
        o->precision != TQR_PRECISION_BF16_UPDATES)
        return -11;
    if (o->reserved != 0) return -11;
    return TQR_OK;
}
// Least squares with the FP64 factorisation (tqr_solve_ls_ex after its
// argument checks): factor, Q^T B, tiled back substitution.
template <int B, int IB>
tqr_status solve_impl(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *Bm, int64_t ldb, double *T,
                      void *work, int32_t *d_info, hipStream_t stream, const tqr_options *po) {
    const Sizes z = sizes_of(m, n, nrhs, B);
    double *W = reinterpret_cast<double *>(work);
    double *Vd = reinterpret_cast<double *>(reinterpret_cast<char *>(work) + z.tiles_bytes);
    double *Bt = reinterpret_cast<double *>(reinterpret_cast<char *>(work) + z.tiles_bytes + z.vd_bytes);
    void *sched = reinterpret_cast<char *>(work) + z.tiles_bytes + z.vd_bytes + z.btiles_bytes;
    // the factorisation's tiles stay in the workspace for the solve
    hipLaunchKernelGGL(k_cm_to_tiles, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, A, lda, m, n, W,
                       (int)z.p, B, B);
    FactorGraph g(z.p, z.q, B);
    const FactorBody<B, IB> body = factor_body<B, IB>(W, T, Vd, z, work, sched, po, stream);
    g.helpers = body.helpers;
    tqr_status s1 = run_graph(g, body, sched, TileKernels<B, IB>::LDS_BYTES, po, stream, po ? po->status : nullptr);
    if (s1 != TQR_OK) return s1;
    hipLaunchKernelGGL(k_tiles_to_cm, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, W, (int)z.p, B, B, A,
                       lda, m, n);
    if (nrhs == 0) return TQR_OK;
    if (narrow_ok(B, IB, nrhs)) {
        // Q^T B and the back substitution in place on B, one workgroup per
        // row tile / row block (tqr_narrow.h)
        const NarrowMem nm = narrow_mem(work, z, B);
        s1 = narrow_apply<B, IB>(true, m, n, nrhs, T, W, Vd, Bm, ldb, nm, stream, po);
        if (s1 != TQR_OK) return s1;
        hipLaunchKernelGGL(k_diag_info, dim3(1), dim3(256), 0, stream, W, (int)z.p, B, n, d_info);
        return narrow_trsv<B>(false, m, n, nrhs, W, Bm, ldb, nm, stream, po);
    }
    s1 = apply_impl<B, IB>(true, m, n, nrhs, T, W, Vd, Bm, ldb, Bt, sched, stream, po);
    if (s1 != TQR_OK) return s1;
    hipLaunchKernelGGL(k_diag_info, dim3(1), dim3(256), 0, stream, W, (int)z.p, B, n, d_info);
    s1 = trsm_impl<B>(m, n, nrhs, W, Bt, sched, stream, po);
    if (s1 != TQR_OK) return s1;
    hipLaunchKernelGGL(k_tiles_to_cm, dim3((unsigned)z.p, 1), dim3(256), 0, stream, Bt, (int)z.p, B, (int)wb_of(nrhs),
                       Bm, ldb, m, nrhs);
    return TQR_OK;
}

// Workspace of the mixed solver: the solve layout (tiles, dense V, B tiles,
// scheduler, progress words, narrow region), then the refinement's vectors
// for one chunk of at most kNarrowRhs right-hand sides: x, p, t, s (n rows),
// r, q (m rows), the partial sums of A t, the per-column state and ||A||_F^2.
struct MixedSizes {
    Sizes z;
    int64_t x, p, t, s, r, q, part, colsq, state, total;
};
inline MixedSizes mixed_sizes(int64_t m, int64_t n, int64_t nrhs, int b) {
    MixedSizes s;
    s.z = sizes_of(m, n, std::min<int64_t>(nrhs, kNarrowRhs), b);
    const int64_t nv = align256(n * kNarrowRhs * 8), mv = align256(m * kNarrowRhs * 8);
    s.x = s.z.total;
    s.p = s.x + nv;
    s.t = s.p + nv;
    s.s = s.t + nv;
    s.r = s.s + nv;
    s.q = s.r + mv;
    s.part = s.q + mv;
    s.colsq = s.part + align256((int64_t)kResidChunks * m * kNarrowRhs * 8);
    s.state = s.colsq + align256(n * 8);
    s.total = s.state + align256((int64_t)kNarrowRhs * (int64_t)sizeof(CglsState) + 64);
    return s;
}

// Mixed-precision least squares (tqr_solve_ls_mixed after its argument
// checks; inner block 16): the factorisation in the requested precision,
// then, for each chunk of at most kNarrowRhs right-hand sides, CGLS in FP64
// on min ||(A R^{-1}) y - b||, x = R^{-1} y, from x = 0 (R, the factor's
// triangle, as a right preconditioner: A R^{-1} is orthogonal up to the
// factor's rounding, so few iterations reach FP64 accuracy).  Every product
// with A and A^T is taken with the caller's FP64 A; the triangular solves use
// the narrow pipelines; the step lengths and the stopping test are computed
// on the device (no host synchronisation).
template <int B>
tqr_status mixed_impl(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *Bm, int64_t ldb,
                      double *X, int64_t ldx, int iterations, double *T, void *work, int32_t *d_info,
                      tqr_refine_stats *stats, hipStream_t stream, const tqr_options &o) {
    const MixedSizes ms = mixed_sizes(std::max<int64_t>(m, 1), std::max<int64_t>(n, 1), nrhs, B);
    const Sizes &z = ms.z;
    char *wbase = reinterpret_cast<char *>(work);
    double *W = reinterpret_cast<double *>(wbase);
    double *Vd = reinterpret_cast<double *>(wbase + z.tiles_bytes);
    void *sched = wbase + z.tiles_bytes + z.vd_bytes + z.btiles_bytes;
    double *xv = reinterpret_cast<double *>(wbase + ms.x), *pv = reinterpret_cast<double *>(wbase + ms.p);
    double *tv = reinterpret_cast<double *>(wbase + ms.t), *sv = reinterpret_cast<double *>(wbase + ms.s);
    double *rv = reinterpret_cast<double *>(wbase + ms.r), *qv = reinterpret_cast<double *>(wbase + ms.q);
    double *part = reinterpret_cast<double *>(wbase + ms.part), *colsq = reinterpret_cast<double *>(wbase + ms.colsq);
    CglsState *st = reinterpret_cast<CglsState *>(wbase + ms.state);
    double *fro2 = reinterpret_cast<double *>(wbase + ms.state + kNarrowRhs * sizeof(CglsState));
    hipLaunchKernelGGL(k_cm_to_tiles, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, A, lda, m, n, W,
                       (int)z.p, B, B);
    FactorGraph g(z.p, z.q, B);
    tqr_status s1;
    if (o.precision == TQR_PRECISION_FP32_UPDATES) {
        const FactorBody<B, 16, true> body = factor_body<B, 16, true>(W, T, Vd, z, work, sched, &o, stream);
        g.helpers = body.helpers;
        s1 = run_graph(g, body, sched, TileKernels<B, 16>::LDS_BYTES, &o, stream, o.status);
    } else if (o.precision == TQR_PRECISION_BF16_UPDATES) {
        const FactorBody<B, 16, true, true> body = factor_body<B, 16, true, true>(W, T, Vd, z, work, sched, &o, stream);
        g.helpers = body.helpers;
        s1 = run_graph(g, body, sched, TileKernels<B, 16>::LDS_BYTES, &o, stream, o.status);
    } else {
        const FactorBody<B, 16> body = factor_body<B, 16>(W, T, Vd, z, work, sched, &o, stream);
        g.helpers = body.helpers;
        s1 = run_graph(g, body, sched, TileKernels<B, 16>::LDS_BYTES, &o, stream, o.status);
    }
    if (s1 != TQR_OK) return s1;
    hipLaunchKernelGGL(k_diag_info, dim3(1), dim3(256), 0, stream, W, (int)z.p, B, n, d_info);
    // ||A||_F^2 (columns, then a fixed-order sum)
    hipLaunchKernelGGL(k_col_sumsq, dim3((unsigned)n), dim3(NT), 0, stream, A, lda, m, colsq);
    hipLaunchKernelGGL(k_sum_vec, dim3(1), dim3(NT), 0, stream, colsq, n, fro2);
    NarrowMem nm = narrow_mem(work, z, B);
    int32_t *done = nm.ints + 4;  // every column of the chunk has stopped
    const unsigned gn4 = (unsigned)cdiv(n * kNarrowRhs, 256), gm4 = (unsigned)cdiv(m * kNarrowRhs, 256);
    for (int64_t c0 = 0; c0 < nrhs; c0 += kNarrowRhs) {
        const int nc = (int)std::min<int64_t>(kNarrowRhs, nrhs - c0);
        // x = 0, r = b, s = R^{-T} A^T b, p = s, gamma = ||s||^2
        hipLaunchKernelGGL(k_copy_cm, dim3(gn4), dim3(256), 0, stream, nullptr, 0, xv, n, n, nc, 0.0);
        hipLaunchKernelGGL(k_copy_cm, dim3(gm4), dim3(256), 0, stream, Bm + c0 * ldb, ldb, rv, m, m, nc, 1.0);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, stream, done, (int64_t)1, 0);
        nm.skip = nullptr;
        hipLaunchKernelGGL(k_gemv_t, dim3((unsigned)n), dim3(NT), 0, stream, A, lda, m, rv, nc, sv, n, nullptr);
        s1 = narrow_trsv<B>(true, m, n, nc, W, sv, n, nm, stream, &o);
        if (s1 != TQR_OK) return s1;
        hipLaunchKernelGGL(k_cgls_start, dim3(nc), dim3(NT), 0, stream, sv, n, pv, rv, m, nc, st, iterations);
        hipLaunchKernelGGL(k_cgls_alldone, dim3(1), dim3(64), 0, stream, st, nc, done);
        // once every column has stopped, the remaining iterations' products
        // and solves return at once (no host synchronisation to cut the loop)
        nm.skip = done;
        for (int it = 0; it < iterations; ++it) {
            // t = R^{-1} p, q = A t, alpha = gamma / ||q||^2, x += alpha t, r -= alpha q
            hipLaunchKernelGGL(k_copy_cm, dim3(gn4), dim3(256), 0, stream, pv, n, tv, n, n, nc, 1.0);
            s1 = narrow_trsv<B>(false, m, n, nc, W, tv, n, nm, stream, &o);
            if (s1 != TQR_OK) return s1;
            hipLaunchKernelGGL(k_resid_partial, dim3((unsigned)cdiv(m, 256), kResidChunks), dim3(256), 0, stream, A,
                               lda, m, n, tv, n, nc, part, done);
            hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)cdiv(m * nc, 256)), dim3(256), 0, stream, part,
                               kResidChunks, m, nc, qv);
            hipLaunchKernelGGL(k_cgls_step, dim3(nc), dim3(NT), 0, stream, qv, m, nc, st);
            hipLaunchKernelGGL(k_cgls_update_xr, dim3((unsigned)cdiv(std::max(m, n) * nc, 256)), dim3(256), 0, stream,
                               xv, tv, n, rv, qv, m, nc, st);
            // residual replacement: r = b - A x in FP64 (the recurrence's r
            // drifts from the true residual by rounding, and the stopping
            // test must see the true one)
            hipLaunchKernelGGL(k_resid_partial, dim3((unsigned)cdiv(m, 256), kResidChunks), dim3(256), 0, stream, A,
                               lda, m, n, xv, n, nc, part, done);
            hipLaunchKernelGGL(k_resid_replace, dim3((unsigned)cdiv(m * nc, 256)), dim3(256), 0, stream, Bm + c0 * ldb,
                               ldb, part, kResidChunks, m, nc, rv, st);
            // s = R^{-T} A^T r, beta = ||s||^2 / gamma, p = s + beta p, stopping test
            hipLaunchKernelGGL(k_gemv_t, dim3((unsigned)n), dim3(NT), 0, stream, A, lda, m, rv, nc, sv, n, done);
            s1 = narrow_trsv<B>(true, m, n, nc, W, sv, n, nm, stream, &o);
            if (s1 != TQR_OK) return s1;
            hipLaunchKernelGGL(k_cgls_next, dim3(nc), dim3(NT), 0, stream, sv, xv, rv, n, m, nc, fro2, st, it + 1);
            hipLaunchKernelGGL(k_cgls_update_p, dim3(gn4), dim3(256), 0, stream, pv, sv, n, nc, st);
            hipLaunchKernelGGL(k_cgls_alldone, dim3(1), dim3(64), 0, stream, st, nc, done);
        }
        hipLaunchKernelGGL(k_copy_cm, dim3(gn4), dim3(256), 0, stream, xv, n, X + c0 * ldx, ldx, n, nc, 1.0);
        if (stats) hipLaunchKernelGGL(k_cgls_report, dim3(1), dim3(64), 0, stream, st, nc, stats + c0);
    }
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

// ---- per (tile_b, inner_ib) pair ------------------------------------------
// The entry points dispatch through this table; each pair's table (and with
// it every kernel the pair instantiates) is defined in a translation unit of
// its own, tqr_inst.hip compiled once per pair.
struct PairFns {
    tqr_status (*factor)(int64_t m, int64_t n, double *A, int64_t lda, double *T, void *work, hipStream_t stream,
                         const tqr_options *opt, bool back_to_cm);
    tqr_status (*apply)(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *T, double *W, const double *Vd,
                        double *Bm, int64_t ldb, double *Bt, void *sched, hipStream_t stream, const tqr_options *opt);
    tqr_status (*solve)(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *Bm, int64_t ldb, double *T,
                        void *work, int32_t *d_info, hipStream_t stream, const tqr_options *po);
    // Q^T / Q on a narrow column-major block (inner block 16 and tile_b 64,
    // 128 or 256 only; null otherwise)
    tqr_status (*apply_narrow)(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *T, const double *W,
                               const double *Vd, double *Bm, int64_t ldb, const NarrowMem &nm, hipStream_t stream,
                               const tqr_options *opt);
    // inner block 16 and tile_b 64, 128 or 256 only; null otherwise
    tqr_status (*mixed)(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *Bm, int64_t ldb,
                        double *X, int64_t ldx, int iterations, double *T, void *work, int32_t *d_info,
                        tqr_refine_stats *stats, hipStream_t stream, const tqr_options &o);
};

template <int B, int IB>
const PairFns &pair_fns();

#define TQR_PAIRS(X) X(16, 16) X(32, 16) X(32, 32) X(64, 16) X(64, 32) X(64, 64) X(128, 16) X(128, 32) X(256, 16) X(256, 32)
#define TQR_DECLARE_PAIR(BB, II) \
    template <>                  \
    const PairFns &pair_fns<BB, II>();
TQR_PAIRS(TQR_DECLARE_PAIR)
#undef TQR_DECLARE_PAIR

}  // namespace tqr
