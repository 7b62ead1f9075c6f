// Host-side builder of a call's launch sequence (internal).
//
// A library call describes its work once through a Program: tile-GEMM jobs with
// their operand segments, interleaved with other kernel launches.  The call runs
// the description twice: a record pass that only collects the GEMM job tables
// (so their size is known and they can be copied to the device in one transfer),
// then an execute pass that launches everything in stream order, pointing each
// GEMM launch at its slice of the uploaded tables.
#pragma once
#include <functional>
#include <mutex>
#include <vector>
#include "common.h"
#include "dag.h"
#include "kernels.h"

namespace gpr {

// Optional event timing of the dominant tile-GEMM launches (a profiling hook of the C-ABI).
struct TimingLog {
  std::mutex mu;
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    double flops;
    int kind;   // timing kind: 0/1 float64/float32 update, 2/3 bf16x3/bf16x6 update,
                // 4/5 float64/float32 inversion step, 6/7 float64/float32 gradient trace,
                // 8/9 bf16x3/bf16x6 inversion step, 10/11 bf16x3/bf16x6 gradient trace
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
inline TimingLog g_timing;

// Host-side access log: what each launch of a description reads and writes (byte ranges
// [lo, hi)), and the event records and waits between the two streams.  Filled by a trace
// pass that launches nothing; check_schedule() (schedule.cpp) uses it to show that
// launches on different streams that touch the same bytes, one of them writing, are
// ordered by events.
struct Span {
  uintptr_t lo, hi;
};
inline Span span(const void* p, size_t bytes) { return Span{(uintptr_t)p, (uintptr_t)p + bytes}; }
// rows x cols elements of esize bytes at p with leading dimension ld (the covering range)
inline Span span2d(const void* p, int64_t rows, int64_t cols, int64_t ld, int esize) {
  if (rows <= 0 || cols <= 0) return Span{(uintptr_t)p, (uintptr_t)p};
  return span(p, (size_t)(((rows - 1) * ld + cols) * esize));
}
struct AccessLog {
  enum { LAUNCH = 0, RECORD = 1, WAIT = 2 };
  struct Op {
    int type, stream, ev;
    std::vector<Span> rd, wr;
  };
  std::vector<Op> ops;
  int64_t unannotated = 0;   // launches issued without access annotations
};
struct ScheduleReport {
  int64_t launches = 0, on_stream[2] = {0, 0}, waits = 0, concurrent_pairs = 0, conflicts = 0, unannotated = 0,
          early_waits = 0;
};
// omit_wait >= 0 analyses the schedule as if the waits on that event were missing.
void check_schedule(const AccessLog& log, int omit_wait, ScheduleReport& rep);

// A task graph recorded from a description (device-side schedule): one task per tile
// product launch or other operation, in issue order, with the byte ranges it reads and
// writes; the edges are derived from those ranges (dag_edges in abi.cpp).
struct DagRecord {
  std::vector<DagTask> tasks;
  std::vector<DagOp> ops;
  std::vector<std::vector<Span>> rd, wr;
  int32_t items = 0;
  int32_t prio = 1;   // ready queue of the tasks recorded next
  bool ok = true;   // false when an operation has no task form (the caller falls back to streams)
  void add(DagTask t, std::vector<Span> r, std::vector<Span> w) {
    t.item0 = items;
    t.prio = prio;
    items += t.nitems;
    tasks.push_back(t);
    rd.push_back(std::move(r));
    wr.push_back(std::move(w));
  }
};

struct Program {
  bool exec = false;
  hipStream_t st = nullptr;        // the caller's stream
  // Look-ahead: a second stream (default priority) and events ordering the two; launches go
  // to the stream selected by on() (0: caller's, 1: auxiliary).  With no events (aux ==
  // st), record() and wait() do nothing and every launch stays in the caller's stream.
  hipStream_t aux = nullptr;
  std::vector<hipEvent_t>* events = nullptr;
  int cur = 0;
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  const GemmJob* djobs = nullptr;
  const GemmSeg* dsegs = nullptr;
  hipError_t err = hipSuccess;
  int64_t gemm_flops_wg = 0;   // workgroups launched (statistics)
  int job0 = 0, nwg = 0, f32 = 0, kind = 0, mt = GEMM_BM;   // mt: macro tile edge of the open launch
  double kind_flops = 0.0;
  bool cur_valid = false;
  // gradient-trace launches: arguments, and running count of their workgroups (each writes
  // three partial sums at partial + 3 * (trace_wg + its block index)); trace_cap bounds it
  const TraceArgs* trace = nullptr;
  int64_t trace_wg = 0, trace_cap = 0;
  AccessLog* alog = nullptr;   // trace pass: log accesses, launch nothing
  DagRecord* dagr = nullptr;   // task-graph pass: record tasks, launch nothing

  hipStream_t stream() const { return cur == 1 && aux ? aux : st; }
  void on(int s) { cur = s; }
  // Event ev is recorded on / waited for by the current stream (execute pass only).
  void record(int ev) {
    if (alog) alog->ops.push_back({AccessLog::RECORD, cur, ev, {}, {}});
    if (!exec || err != hipSuccess || !events || ev >= (int)events->size()) return;
    err = hipEventRecord((*events)[ev], stream());
  }
  void wait(int ev) {
    if (alog) alog->ops.push_back({AccessLog::WAIT, cur, ev, {}, {}});
    if (!exec || err != hipSuccess || !events || ev >= (int)events->size()) return;
    err = hipStreamWaitEvent(stream(), (*events)[ev], 0);
  }

  void reset_for_exec(const GemmJob* dj, const GemmSeg* ds) {
    exec = true;
    djobs = dj;
    dsegs = ds;
    jobs.clear();
    segs.clear();
  }
  size_t table_bytes() const { return jobs.size() * sizeof(GemmJob) + segs.size() * sizeof(GemmSeg) + 512; }

  // `algo_flops` is the launch's algorithmic flop count (used by the timing hook).
  void gemm_begin(int use_f32, int launch_kind = 0, double algo_flops = 0.0) {
    job0 = (int)jobs.size();
    nwg = 0;
    f32 = use_f32;
    kind = launch_kind;
    mt = gemm_kind_macro(launch_kind);
    kind_flops = algo_flops;
  }
  // Adds a job C[M x N] = alpha * sum(segments added next) + beta * Cin.
  void job(void* C, int64_t ldc, const void* Cin, int64_t ldcin, int64_t M, int64_t N, double alpha, double beta,
           int flags, int aux0 = 0, int aux1 = 0) {
    GemmJob j{};
    j.C = C;
    j.Cin = Cin;
    j.ldc = ldc;
    j.ldcin = ldcin;
    j.alpha = alpha;
    j.beta = beta;
    j.M = (int32_t)M;
    j.N = (int32_t)N;
    j.seg0 = (int32_t)segs.size();
    j.nseg = 0;
    j.wg_begin = nwg;
    j.tiles_n = (int32_t)ceil_div(N, mt);
    j.flags = flags;
    j.aux0 = aux0;
    j.aux1 = aux1;
    cur_valid = M > 0 && N > 0;
    if (!cur_valid) return;
    const int64_t tiles = ceil_div(M, mt) * (int64_t)j.tiles_n;
    jobs.push_back(j);
    nwg += (int)tiles;
  }
  void seg(const void* A, int64_t lda, int modeA, const void* B, int64_t ldb, int modeB, int64_t K, int tri = 0) {
    if (!cur_valid || K <= 0) return;
    GemmSeg s{};
    s.A = A;
    s.B = B;
    s.lda = lda;
    s.ldb = ldb;
    s.K = (int32_t)K;
    s.modeA = (uint8_t)modeA;
    s.modeB = (uint8_t)modeB;
    s.tri = (uint8_t)tri;
    segs.push_back(s);
    jobs.back().nseg++;
  }
  void gemm_end() {
    const int nj = (int)jobs.size() - job0;
    if (alog && nj > 0) log_gemm(nj);
    if (dagr) {
      if (nj == 0) return;
      if (f32 || gemm_kind_trace(kind) || gemm_kind_macro(kind) != GEMM_BM || kind == GEMM_KIND_WIDEN ||
          gemm_kind_bf16(kind)) {
        dagr->ok = false;   // the task form covers the float64 tile products only
        return;
      }
      DagTask t{};
      t.kind = DAG_GEMM;
      t.spec = gemm_launch_spec(jobs.data() + job0, nj, segs.data(), 8, 16);
      t.nitems = nwg;
      t.job0 = job0;
      t.njobs = nj;
      std::vector<Span> rd, wr;
      gemm_spans(nj, rd, wr);
      dagr->add(t, std::move(rd), std::move(wr));
      return;
    }
    if (!exec || err != hipSuccess || nj == 0) return;
    gemm_flops_wg += nwg;
    hipEvent_t ea = nullptr, eb = nullptr;
    bool timed = false;
    if (kind == GEMM_KIND_UPDATE || (gemm_kind_bf16(kind) && !gemm_kind_solve(kind)) || gemm_kind_trtri(kind) ||
        gemm_kind_trace(kind)) {
      std::lock_guard<std::mutex> lk(g_timing.mu);
      if (g_timing.on) {
        ea = g_timing.get();
        eb = g_timing.get();
        timed = ea && eb;
      }
    }
    hipStream_t sx = stream();
    if (gemm_kind_macro(kind) == 256) {
      // the 256 x 256 kernel has no bounds checks: whole macro tiles, 16-deep chunks and
      // tiled-layout planes whose row length is the segment depth
      for (int jx = job0; jx < job0 + nj; ++jx) {
        const GemmJob& J = jobs[jx];
        bool ok = J.M % 256 == 0 && J.N % 256 == 0;
        for (int sx2 = J.seg0; ok && sx2 < J.seg0 + J.nseg; ++sx2) {
          const GemmSeg& S = segs[sx2];
          ok = S.K % 16 == 0 && S.lda == S.K && S.ldb == S.K && S.modeA == MODE_KC && S.modeB == MODE_KC &&
               S.tri == 0;
        }
        if (!ok) {
          err = hipErrorInvalidValue;
          return;
        }
      }
    }
    if (gemm_kind_trace(kind) && (!trace || trace_wg + nwg > trace_cap)) {
      err = hipErrorInvalidValue;
      return;
    }
    const int esize = (f32 || kind == GEMM_KIND_WIDEN) ? 4 : 8;
    const int bk = 16;   // chunk depth of the main loop (both product types)
    const int spec = gemm_kind_bf16(kind) ? -1 : gemm_launch_spec(jobs.data() + job0, nj, segs.data(), esize, bk);
    if (timed) (void)hipEventRecord(ea, sx);
    if (gemm_kind_trace(kind)) {
      TraceArgs ta = *trace;
      ta.partial += 3 * trace_wg;
      err = gemm_kind_bf16(kind) ? launch_gemm_bf16_trace_t256(gemm_kind_nprod(kind), djobs + job0, dsegs, nj, nwg, ta, sx)
                                 : launch_gemm_trace(f32, djobs + job0, dsegs, nj, nwg, spec, ta, sx);
      trace_wg += nwg;
    } else {
      err = launch_gemm(f32, djobs + job0, dsegs, nj, nwg, kind, spec, sx);
    }
    if (timed) {
      (void)hipEventRecord(eb, sx);
      std::lock_guard<std::mutex> lk(g_timing.mu);
      int tk = f32 ? 1 : 0;
      const int six = gemm_kind_nprod(kind) == 6 ? 1 : 0;
      if (gemm_kind_bf16(kind)) tk = gemm_kind_trtri(kind) ? 8 + six : (gemm_kind_trace(kind) ? 10 + six : 2 + six);
      else if (kind == GEMM_KIND_TRTRI) tk = f32 ? 5 : 4;
      else if (kind == GEMM_KIND_TRACE) tk = f32 ? 7 : 6;
      g_timing.recs.push_back({ea, eb, kind_flops, tk});
    }
  }
  // Launches produced by `fn` (given the current stream) run only in the execute pass.
  // `rd` / `wr`: the byte ranges the launch reads / writes (read-modify-write counts as a
  // write), for the trace pass.
  void kernel(const std::function<hipError_t(hipStream_t)>& fn) {
    if (dagr) {
      dagr->ok = false;
      return;
    }
    if (alog) {
      alog->ops.push_back({AccessLog::LAUNCH, cur, -1, {}, {}});
      alog->unannotated++;
    }
    if (!exec || err != hipSuccess) return;
    err = fn(stream());
  }
  void kernel(const std::function<hipError_t(hipStream_t)>& fn, std::vector<Span> rd, std::vector<Span> wr) {
    if (dagr) {
      dagr->ok = false;
      return;
    }
    if (alog) alog->ops.push_back({AccessLog::LAUNCH, cur, -1, std::move(rd), std::move(wr)});
    if (!exec || err != hipSuccess) return;
    err = fn(stream());
  }

  // An operation other than a tile product: launched by `fn` (streams), or recorded as a
  // task of `nitems` items described by `d` (task-graph pass).
  void op(int dag_kind, const DagOp& d, int64_t nitems, const std::function<hipError_t(hipStream_t)>& fn,
          std::vector<Span> rd, std::vector<Span> wr) {
    if (dagr) {
      if (nitems <= 0) return;
      DagTask t{};
      t.kind = dag_kind;
      t.nitems = (int32_t)nitems;
      t.op = (int32_t)dagr->ops.size();
      dagr->ops.push_back(d);
      dagr->add(t, std::move(rd), std::move(wr));
      return;
    }
    kernel(fn, std::move(rd), std::move(wr));
  }

  // Access ranges of the open tile-GEMM launch: C (and Cin) of every job, the operand
  // extents of its segments (all planes in the split modes).
  void log_gemm(int nj) {
    AccessLog::Op op{AccessLog::LAUNCH, cur, -1, {}, {}};
    gemm_spans(nj, op.rd, op.wr);
    alog->ops.push_back(std::move(op));
  }
  void gemm_spans(int nj, std::vector<Span>& rd, std::vector<Span>& wr) const {
    struct {
      std::vector<Span>& rd;
      std::vector<Span>& wr;
    } op{rd, wr};
    const bool split = gemm_kind_bf16(kind);
    const int oe = split ? 2 : ((f32 || kind == GEMM_KIND_WIDEN) ? 4 : 8);
    const int planes = split ? (gemm_kind_nprod(kind) == 6 ? 3 : 2) : 1;
    for (int jx = job0; jx < job0 + nj; ++jx) {
      const GemmJob& J = jobs[jx];
      const int ce = (J.flags & JOB_C_F32) ? 4 : 8;
      op.wr.push_back(span2d(J.C, J.M, J.N, J.ldc, ce));
      if (J.Cin && J.beta != 0.0) op.rd.push_back(span2d(J.Cin, J.M, J.N, J.ldcin, ce));
      for (int sx = J.seg0; sx < J.seg0 + J.nseg; ++sx) {
        const GemmSeg& S = segs[sx];
        for (int p = 0; p < planes; ++p) {
          const char* a = (const char*)S.A + (size_t)p * S.pstrideA * oe;
          const char* bp = (const char*)S.B + (size_t)p * S.pstrideB * oe;
          op.rd.push_back(S.modeA == MODE_KC ? span2d(a, J.M, S.K, S.lda, oe) : span2d(a, S.K, J.M, S.lda, oe));
          op.rd.push_back(S.modeB == MODE_KC ? span2d(bp, J.N, S.K, S.ldb, oe) : span2d(bp, S.K, J.N, S.ldb, oe));
        }
      }
    }
  }
};

}  // namespace gpr
