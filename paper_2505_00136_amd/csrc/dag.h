// Device-side task-graph scheduling of the tiled factorisation (internal).
//
// The tasks of Fig. 1 (POTRF, TRSM, SYRK, GEMM) and the steps inside them become a graph
// whose edges are the dependencies between the tiles they read and write; a persistent
// kernel executes it.  A task whose predecessors have all finished is appended to one of
// two ready queues (the critical path of the factorisation -- diagonal tile, panel, the
// next block column's update -- in the first, which is always served first); workgroups
// take the next work item of the oldest task of a queue that still has items, run it, and
// the workgroup that finishes a task's last item decrements its successors' counters and
// appends those that reach zero.  A workgroup never waits while holding an item, so no
// workgroup can block another, whatever number is resident.  This takes the place of the
// futures and dataflow of the paper's runtime (Sections 3.1 and 4.2).
//
// The scheduling logic (claim, finish, the give-up rule) is written once against an
// atomics policy so that the host runs exactly this code with threads in its tests
// (gpr_dag_check) and the device with agent-scope atomics (dag.hip).
#pragma once
#include <stdint.h>

#include "common.h"

#define GPR_HD __host__ __device__

namespace gpr {

enum { DAG_GEMM = 0, DAG_POTRF = 1, DAG_IDENTITY = 2, DAG_ZERO_UPPER = 3, DAG_COPY = 4, DAG_TRANSPOSE = 5 };

// A task: `nitems` work items that may start once its `npred` predecessor tasks have finished.
struct DagTask {
  int32_t kind;           // DAG_*
  int32_t spec;           // DAG_GEMM: main-loop specialisation (gemm_launch_spec)
  int32_t item0, nitems;  // its items (item0: running count in issue order, for reference)
  int32_t npred;          // predecessor tasks
  int32_t succ0, nsucc;   // successors: succ[succ0 .. succ0 + nsucc)
  int32_t job0, njobs;    // DAG_GEMM: its jobs in the job table (job wg_begin counts from the task's first item)
  int32_t op;             // other kinds: index into the op table
  int32_t prio;           // ready queue: 0 (critical path, served first) or 1
};

// Parameters of a task that is not a tile product.
//   DAG_POTRF:      p0 = A (diagonal block), p1 = W (its inverse), i0 = lda = ldw, i1 = jb, i2 = global column of A(0,0)
//   DAG_IDENTITY:   p0 = W (b x b float64), i0 = b         (items of 4096 elements)
//   DAG_ZERO_UPPER: p0 = A (b x b float64), i0 = b         (items of 4096 elements)
//   DAG_COPY:       p0 = dst, p1 = src, i0 = bytes          (16-byte aligned; items of 128 KiB)
//   DAG_TRANSPOSE:  p0 = dst, p1 = src, i0 = b, i1 = tiles, i2 = element bytes (items: 64 x 64 blocks)
struct DagOp {
  void* p0;
  const void* p1;
  int64_t i0, i1, i2, i3;
};

struct DagCtl {
  int32_t head[2];      // oldest task of each ready queue that may still have items
  int32_t tail[2];      // slots handed out in each ready queue
  int32_t finished;     // finished tasks
  int32_t abort;        // raised when no task finished for longer than the time limit
  int32_t timed_out;    // workgroups that gave up
  int32_t pad;
};

// Items of a task are handed out in DAG_LANES contiguous lanes, one per XCD of the device
// (the CDNA4 chip has eight, each with its own L2): a workgroup takes items from the lane
// of its own XCD first, so neighbouring macro tiles that share operand rows run on the
// same L2, and takes from the other lanes once its own is empty.
constexpr int DAG_LANES = 8;

// Device state of one graph run: per task the unfinished predecessors, the unfinished
// items, the next item of each lane, and the two ready queues (-1: slot not written yet).
// The lane counters are stored lane by lane, so that the workgroups of different XCDs
// claiming items of one task increment counters in different cache lines.
struct DagState {
  int32_t *pending, *remaining, *next_item, *rq0, *rq1;
  DagCtl* ctl;
  int32_t ntasks;
};
inline size_t dag_state_ints(int64_t ntasks) { return (4 + DAG_LANES) * (size_t)ntasks + 64; }
GPR_HD inline DagState dag_state_at(int32_t* base, int32_t ntasks) {
  DagState S;
  S.pending = base;
  S.remaining = base + ntasks;
  S.rq0 = base + 2 * (size_t)ntasks;
  S.rq1 = base + 3 * (size_t)ntasks;
  S.next_item = base + 4 * (size_t)ntasks;   // [lane][task]: each lane's counters in lines of their own
  S.ctl = (DagCtl*)(base + (((4 + DAG_LANES) * (size_t)ntasks + 15) & ~(size_t)15));
  S.ntasks = ntasks;
  return S;
}

constexpr int64_t DAG_ELEMS_PER_ITEM = 4096;
// pivot word left by a graph whose executor gave up (no pivot column is this large)
constexpr unsigned long long DAG_ABORT_INFO = 0x7ffffffffffffffeull;
constexpr int64_t DAG_COPY_BYTES_PER_ITEM = 128 * 1024;

// Memory ordering: a task's results are made visible by the workgroups that wrote them
// (each finishes an item with a release decrement of the task's item counter); the last
// finisher acquires them all (an acquire fence after the decrement that reached zero) and
// passes them on with release decrements of its successors' counters; the decrement that
// brings a successor to zero is followed by an acquire fence and the release store that
// publishes it.  A consumer reads queue slots and counters with relaxed device-scope
// atomics (coherent across XCDs, no cache invalidation) and runs an item only after an
// acquire fence that follows the publication of the item's task; the executor skips that
// fence when its previous one already did (ready-queue slots handed out before the fence).
template <class Ops>
struct DagCore {
  // Appends task t to its ready queue (after its last predecessor finished).
  static GPR_HD void publish(const DagTask* tasks, DagState& S, int t) {
    const int q = tasks[t].prio ? 1 : 0;
    const int slot = Ops::fetch_add_relaxed(&S.ctl->tail[q], 1);
    Ops::store_release(q ? &S.rq1[slot] : &S.rq0[slot], t);
  }

  // The next item of a ready task for a workgroup on lane x: true with (t, idx) and the
  // queue q and slot h it came from, false when no ready task has items left right now.
  // Queue 0 first; within a queue the oldest task that still has items; within the task
  // the lane x first.
  static GPR_HD bool try_claim(const DagTask* tasks, DagState& S, int x, int& t, int& idx, int& q, int& h) {
    for (q = 0; q < 2; ++q) {
      int32_t* rq = q ? S.rq1 : S.rq0;
      h = Ops::load_relaxed(&S.ctl->head[q]);
      while (h < Ops::load_relaxed(&S.ctl->tail[q])) {
        const int tt = Ops::load_relaxed(&rq[h]);
        if (tt < 0) break;   // the slot is handed out but not written yet: look again later
        const int n = tasks[tt].nitems;
        for (int c = 0; c < DAG_LANES; ++c) {
          const int lane = (x + c) % DAG_LANES;
          const int lo = (int)((int64_t)n * lane / DAG_LANES), hi = (int)((int64_t)n * (lane + 1) / DAG_LANES);
          if (lo >= hi) continue;
          const int i = Ops::fetch_add_relaxed(&S.next_item[(size_t)lane * S.ntasks + tt], 1);
          if (lo + i < hi) {
            t = tt;
            idx = lo + i;
            return true;
          }
        }
        // the task has no items left: move the head past it (another may already have)
        Ops::cas_relaxed(&S.ctl->head[q], h, h + 1);
        h = Ops::load_relaxed(&S.ctl->head[q]);
      }
    }
    return false;
  }

  // After an item of task t has finished and its results are visible to this thread: the
  // last item of the task releases its successors, publishing those with no unfinished
  // predecessor left.
  static GPR_HD void finish(const DagTask* tasks, const int32_t* succ, DagState& S, int t) {
    if (Ops::fetch_add_release(&S.remaining[t], -1) != 1) return;
    Ops::fence_acquire();   // the other items' results
    const DagTask& T = tasks[t];
    for (int q = 0; q < T.nsucc; ++q) {
      const int s = succ[T.succ0 + q];
      if (Ops::fetch_add_release(&S.pending[s], -1) == 1) {
        Ops::fence_acquire();   // the other predecessors' results
        publish(tasks, S, s);
      }
    }
    Ops::fetch_add_release(&S.ctl->finished, 1);
  }

  // The give-up rule for a workgroup that found nothing to claim: false (stop) once every
  // task has finished, the abort flag is up, or no task has finished for `limit` clock
  // ticks (then the flag is raised); `last` and `since` carry the progress it last saw.
  static GPR_HD bool keep_waiting(DagState& S, int& last, uint64_t& since, uint64_t limit) {
    const int f = Ops::load_relaxed(&S.ctl->finished);
    if (f >= S.ntasks) return false;
    if (Ops::load_relaxed(&S.ctl->abort) != 0) return false;
    const uint64_t now = Ops::clock();
    if (f != last) {
      last = f;
      since = now;
    } else if (now - since > limit) {
      Ops::fetch_add_relaxed(&S.ctl->timed_out, 1);
      Ops::store_release(&S.ctl->abort, 1);
      return false;
    }
    Ops::pause();
    return true;
  }
};

}  // namespace gpr
