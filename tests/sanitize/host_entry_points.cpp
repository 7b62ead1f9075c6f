// Host-only entry points of libgpr driven under AddressSanitizer and UndefinedBehaviorSanitizer
// (the library's host code built with both; no GPU is touched): sizing calls over a grid of
// shapes including empty, ragged and invalid ones, the task census, the happens-before check of
// the stream schedules with and without each wait, and the host model of the device task graph
// with several thread counts, a withheld dependency and dropped edges.  Exits non-zero when a
// result differs from what the library documents; the sanitizers abort on any memory error or
// undefined behaviour.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "gpr.h"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

int main() {
  EXPECT(gpr_version() > 0);
  const int precs[] = {GPR_FP64, GPR_FP32, GPR_BF16X6, GPR_BF16X3};
  // sizing: every shape either sizes or reports an argument error
  const int64_t ns[] = {0, 1, 2, 7, 64, 100, 1000, 4097};
  const int64_t tiles[] = {1, 3, 64, 100, 256, 5000};
  for (int prec : precs)
    for (int64_t n : ns)
      for (int64_t t : tiles) {
        if ((n + t - 1) / t > 40) continue;   // keep the descriptions small
        size_t tb = 0, wb = 0;
        EXPECT(gpr_tiles_bytes(n, t, prec, &tb) == GPR_OK);
        EXPECT(gpr_workspace_size(n, 33, 5, t, prec, &wb) == GPR_OK);
      }
  size_t bytes = 0;
  EXPECT(gpr_tiles_bytes(-1, 64, GPR_FP64, &bytes) != GPR_OK);
  EXPECT(gpr_tiles_bytes(64, 0, GPR_FP64, &bytes) != GPR_OK);
  EXPECT(gpr_tiles_bytes(64, 64, 99, &bytes) != GPR_OK);
  EXPECT(gpr_workspace_size(64, -2, 3, 64, GPR_FP64, &bytes) != GPR_OK);
  EXPECT(gpr_set_schedule(7) != GPR_OK);
  EXPECT(gpr_last_error() != nullptr);
  EXPECT(gpr_mlp_nparams() > 0);
  EXPECT(gpr_mlp_workspace(128, &bytes) == GPR_OK && bytes > 0);
  EXPECT(gpr_stats_workspace(1000, &bytes) == GPR_OK);
  // task census of Fig. 1
  std::vector<int64_t> counts(16, 0);
  for (int64_t T = 1; T <= 40; ++T) EXPECT(gpr_cholesky_census(T, counts.data()) == GPR_OK);
  // happens-before check of the two-stream schedule: no conflict with all waits, and
  // dropping the waits on one event leaves a conflict
  for (int prec : precs)
    for (int64_t T : {1, 2, 3, 5, 9}) {
      int64_t rep[8] = {0};
      EXPECT(gpr_cholesky_schedule_check(T * 64, 64, prec, -1, rep) == GPR_OK);
      EXPECT(rep[5] == 0);
      if (T >= 3) {
        EXPECT(gpr_cholesky_schedule_check(T * 64, 64, prec, 2, rep) == GPR_OK);   // block column 1 updated
        EXPECT(rep[5] > 0);
      }
    }
  // host model of the device task graph
  for (int64_t n : {64, 700, 1000, 3000})
    for (int threads : {1, 4, 16}) {
      int64_t rep[9] = {0};
      EXPECT(gpr_dag_check(n, n < 1000 ? 64 : 256, threads, -1, 10000.0, rep) == GPR_OK);
      EXPECT(rep[3] == rep[1] && rep[4] == 0 && rep[5] == 0 && rep[7] == threads && rep[8] == 0);
    }
  {
    int64_t rep[9] = {0};
    EXPECT(gpr_dag_check(1024, 256, 8, 17, 50.0, rep) == GPR_OK);
    EXPECT(rep[5] == 1 && rep[7] == 8 && rep[3] < rep[1]);
    EXPECT(gpr_dag_check(1024, 256, 2, -2 - 5, 10000.0, rep) == GPR_OK);
  }
  std::printf("host entry points: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
