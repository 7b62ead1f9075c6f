// Happens-before check of a recorded two-stream schedule (host only).
//
// The tiled factorisation's task dependencies (Fig. 1: POTRF(k) after the updates of
// tile (k,k), TRSM(m,k) after POTRF(k) and the updates of tile (m,k), the updates of
// tile (m,n) at step k after TRSM(m,k) and TRSM(n,k), updates of one tile in ascending k)
// are all read-after-write, write-after-read or write-after-write hazards on tile
// memory.  Launches on one stream run in issue order; launches on different streams are
// ordered only through an event recorded on one and waited for on the other.  The check
// replays the log with vector clocks and reports every pair of launches on different
// streams that is ordered in neither direction while one writes bytes the other reads or
// writes.
#include <algorithm>
#include "program.h"

namespace gpr {

namespace {

constexpr int kStreams = 2;

struct Launch {
  int stream;
  int64_t seq;                 // 1-based position among the launches of its stream
  int64_t vc[kStreams];        // launches of each stream known to precede it
  std::vector<Span> rd, wr;    // sorted, merged
};

std::vector<Span> merged(std::vector<Span> v) {
  v.erase(std::remove_if(v.begin(), v.end(), [](const Span& s) { return s.hi <= s.lo; }), v.end());
  std::sort(v.begin(), v.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
  std::vector<Span> out;
  for (const Span& s : v) {
    if (!out.empty() && s.lo <= out.back().hi) out.back().hi = std::max(out.back().hi, s.hi);
    else out.push_back(s);
  }
  return out;
}

bool overlaps(const std::vector<Span>& a, const std::vector<Span>& b) {
  size_t i = 0, j = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i].hi <= b[j].lo) ++i;
    else if (b[j].hi <= a[i].lo) ++j;
    else return true;
  }
  return false;
}

// a precedes b (a, b on different streams)
bool precedes(const Launch& a, const Launch& b) { return a.seq <= b.vc[a.stream]; }

}  // namespace

void check_schedule(const AccessLog& log, int omit_wait, ScheduleReport& rep) {
  rep = ScheduleReport{};
  rep.unannotated = log.unannotated;
  int64_t vc[kStreams][kStreams] = {};
  std::vector<std::vector<int64_t>> ev_vc;
  std::vector<bool> ev_set;
  std::vector<Launch> launches;
  for (const AccessLog::Op& op : log.ops) {
    const int s = op.stream;
    if (s < 0 || s >= kStreams) continue;
    if (op.type == AccessLog::LAUNCH) {
      Launch L{};
      L.stream = s;
      L.seq = ++vc[s][s];
      for (int t = 0; t < kStreams; ++t) L.vc[t] = vc[s][t];
      L.rd = merged(op.rd);
      L.wr = merged(op.wr);
      launches.push_back(std::move(L));
      rep.launches++;
      rep.on_stream[s]++;
    } else if (op.type == AccessLog::RECORD) {
      if (op.ev >= (int)ev_vc.size()) {
        ev_vc.resize(op.ev + 1, std::vector<int64_t>(kStreams, 0));
        ev_set.resize(op.ev + 1, false);
      }
      for (int t = 0; t < kStreams; ++t) ev_vc[op.ev][t] = vc[s][t];
      ev_set[op.ev] = true;
    } else if (op.type == AccessLog::WAIT) {
      rep.waits++;
      if (op.ev == omit_wait) continue;
      // waiting for an event that was never recorded does not wait
      if (op.ev >= (int)ev_set.size() || !ev_set[op.ev]) {
        rep.early_waits++;
        continue;
      }
      for (int t = 0; t < kStreams; ++t) vc[s][t] = std::max(vc[s][t], ev_vc[op.ev][t]);
    }
  }
  std::vector<const Launch*> by[kStreams];
  for (const Launch& L : launches) by[L.stream].push_back(&L);
  for (const Launch* a : by[0])
    for (const Launch* b : by[1]) {
      if (precedes(*a, *b) || precedes(*b, *a)) continue;
      rep.concurrent_pairs++;
      if (overlaps(a->wr, b->wr) || overlaps(a->wr, b->rd) || overlaps(a->rd, b->wr)) rep.conflicts++;
    }
}

}  // namespace gpr
