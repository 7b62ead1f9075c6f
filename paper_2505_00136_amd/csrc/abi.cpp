// C-ABI entry points (include/gpr.h): argument checks, workspace carving and the
// launch sequences of each step of the GP hot path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <unordered_map>
#include <mutex>
#include <string>
#include <chrono>
#include <thread>
#include <vector>

#include "gpr.h"
#include "common.h"
#include "kernels.h"
#include "program.h"

using namespace gpr;

namespace {

thread_local char g_err[512] = "no error";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(GPR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// diagonal-block edge of the in-tile factorisation (set from the environment for tuning runs only)
constexpr int64_t kInnerBlock = 64;     // block edge of the in-tile factorisation loop
constexpr int64_t kRowsPerChunk = 256;  // rows per workgroup of the transposed matrix-vector products
constexpr int64_t kColsPerChunk = 4096; // training points per workgroup of the fused kernel-vector products
constexpr int GPR_BF16X3_SWEEPS = 6;    // default refinement sweeps of the three-product split

bool is_mixed(int prec) { return prec != GPR_FP64; }
// Refinement sweeps of gpr_solve (refine_sweeps < 0) and gpr_optimize per precision: none
// in float64; with a factor of unit roundoff u each sweep contracts the error of alpha by
// about kappa u, so the split-bfloat16 mode with three products (u ~ 2^-16) needs more
// sweeps than float32 and bf16x6 (u ~ 2^-24) to reach the same accuracy.
int default_sweeps(int prec) {
  return prec == GPR_FP64 ? 0 : (prec == GPR_BF16X3 ? GPR_BF16X3_SWEEPS : 3);
}
bool is_bf16(int prec) { return prec == GPR_BF16X3 || prec == GPR_BF16X6; }
int esize_of(int prec) { return is_mixed(prec) ? 4 : 8; }

int check_prec(int prec) {
  if (prec < GPR_FP64 || prec > GPR_BF16X6) return fail(GPR_ERR_ARG, "unknown precision tag %d", prec);
  return GPR_OK;
}

int check_shape(int64_t n, int64_t tile) {
  if (n < 0) return fail(GPR_ERR_SHAPE, "negative size n=%lld", (long long)n);
  if (tile < 1) return fail(GPR_ERR_SHAPE, "tile must be >= 1 (got %lld)", (long long)tile);
  if (tile > (int64_t)1 << 20 || n > (int64_t)1 << 24)
    return fail(GPR_ERR_OOM, "size too large (n=%lld, tile=%lld)", (long long)n, (long long)tile);
  return GPR_OK;
}

int check_hyper(const gpr_hyper_t& h) {
  if (!std::isfinite(h.lengthscale) || !(h.lengthscale > 0.0)) return fail(GPR_ERR_ARG, "lengthscale must be finite and > 0");
  if (!std::isfinite(h.signal_var) || !(h.signal_var > 0.0)) return fail(GPR_ERR_ARG, "signal_var must be finite and > 0");
  if (!std::isfinite(h.noise_var) || h.noise_var < 0.0) return fail(GPR_ERR_ARG, "noise_var must be finite and >= 0");
  if (h.kernel < GPR_KERNEL_SE || h.kernel > GPR_KERNEL_MATERN52) return fail(GPR_ERR_ARG, "unknown kernel %d", h.kernel);
  return GPR_OK;
}

static_assert(GPR_KERNEL_SE == KERNEL_SE && GPR_KERNEL_MATERN12 == KERNEL_M12 && GPR_KERNEL_MATERN32 == KERNEL_M32 &&
                  GPR_KERNEL_MATERN52 == KERNEL_M52, "kernel tags of the C-ABI and the device code differ");

HyperArg harg(const gpr_hyper_t& h) { return HyperArg{h.lengthscale, h.signal_var, h.noise_var, nullptr, h.kernel}; }

TileLayout layout_of(int64_t n, int64_t tile, int prec) {
  TileLayout L;
  L.n = n;
  L.b = tile;
  L.T = tile > 0 ? (n + tile - 1) / tile : 0;
  L.esize = esize_of(prec);
  return L;
}

// Symbolic addresses for the passes that only size or analyse a description (no memory
// behind them): the tiled matrix, the workspace and an output, far apart.
void* const kSymK = (void*)((uintptr_t)1 << 40);
void* const kSymOut = (void*)((uintptr_t)1 << 43);
void* const kSymWs = (void*)((uintptr_t)1 << 46);

// Sequential carving of a workspace into 256-byte aligned regions.  With a null base it
// only sizes (the regions are then null too: no arithmetic on a null pointer).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Per-device resources, created by gpr_init (or, for a device gpr_init did not cover, by
// the first call that needs them) and kept for the life of the process:
//  - the look-ahead's auxiliary stream (default priority, non-blocking) and its events;
//  - a ring of pinned staging slots for the job-table uploads.  Each slot is guarded by
//    the event recorded after its copy, so a call waits only when the ring wraps onto a
//    slot whose copy the GPU has not reached yet (kStageSlots uploads in flight).  A slot
//    smaller than a call's tables is re-allocated, which gpr_init avoids by sizing the
//    slots for the largest problem up front.
constexpr int kMaxDevices = 64;
constexpr int kStageSlots = 8;
constexpr size_t kMinSlotBytes = (size_t)1 << 20;

struct StageSlot {
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool inflight = false;
};

struct DevRes {
  std::mutex mu;        // staging ring, stream and event pool
  std::mutex chol_mu;   // factorisations that use the auxiliary stream and its events
  hipStream_t aux = nullptr;
  std::vector<hipEvent_t> events;
  StageSlot slot[kStageSlots];
  int next = 0;
  int dag_slots = 0;    // workgroups of the task-graph executor that fit at once (0: not queried yet)
};
DevRes g_res[kMaxDevices];

int current_res(DevRes** r) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GPR_ERR_HIP, "device %d out of range", dev);
  *r = &g_res[dev];
  return GPR_OK;
}

// Grows every staging slot to `bytes` (R->mu held); waits for a slot's copy before freeing it.
int grow_slots(DevRes* R, size_t bytes) {
  bytes = std::max(bytes, kMinSlotBytes);
  for (StageSlot& s : R->slot) {
    if (!s.ev) HIPCHK(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    if (s.cap >= bytes) continue;
    if (s.inflight) HIPCHK(hipEventSynchronize(s.ev));
    s.inflight = false;
    if (s.host) HIPCHK(hipHostFree(s.host));
    s.host = nullptr;
    s.cap = 0;
    HIPCHK(hipHostMalloc((void**)&s.host, bytes, hipHostMallocDefault));
    s.cap = bytes;
  }
  return GPR_OK;
}

// Auxiliary stream and at least `nevents` events of the current device (R->mu held).
int ensure_aux(DevRes* R, int nevents) {
  if (!R->aux) HIPCHK(hipStreamCreateWithFlags(&R->aux, hipStreamNonBlocking));
  while ((int)R->events.size() < nevents) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    R->events.push_back(e);
  }
  return GPR_OK;
}

size_t jobs_part(size_t nj) { return (nj * sizeof(GemmJob) + 255) & ~(size_t)255; }

size_t arena_bytes_of(const Program& P) { return jobs_part(P.jobs.size()) + P.segs.size() * sizeof(GemmSeg) + 1024; }

// Uploads the job and segment tables of P into `arena` (jobs first, segments at a
// 256-byte boundary) through the next staging slot; returns the device addresses.
int upload_tables(const Program& P, void* arena, size_t cap, hipStream_t st, const GemmJob** dj, const GemmSeg** ds) {
  const size_t jp = jobs_part(P.jobs.size());
  const size_t bytes = jp + P.segs.size() * sizeof(GemmSeg);
  if (bytes + 1024 > cap) return fail(GPR_ERR_WORKSPACE, "job-table arena too small (%zu > %zu)", bytes + 1024, cap);
  *dj = (const GemmJob*)arena;
  *ds = (const GemmSeg*)((char*)arena + jp);
  if (bytes == 0) return GPR_OK;
  DevRes* R = nullptr;
  int rc = current_res(&R);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(R->mu);
  if (R->slot[R->next].cap < bytes && (rc = grow_slots(R, bytes * 2))) return rc;
  StageSlot& s = R->slot[R->next];
  R->next = (R->next + 1) % kStageSlots;
  if (!s.ev) HIPCHK(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
  if (s.inflight) HIPCHK(hipEventSynchronize(s.ev));   // the ring wrapped onto a copy still queued
  if (!P.jobs.empty()) memcpy(s.host, P.jobs.data(), P.jobs.size() * sizeof(GemmJob));
  if (!P.segs.empty()) memcpy(s.host + jp, P.segs.data(), P.segs.size() * sizeof(GemmSeg));
  HIPCHK(hipMemcpyAsync(arena, s.host, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(s.ev, st));
  s.inflight = true;
  return GPR_OK;
}

// Uploads host arrays into `arena`, each at a 256-byte boundary, through the next staging
// slot (one copy); their device addresses are returned in `dev`.
int upload_parts(const std::vector<std::pair<const void*, size_t>>& parts, void* arena, size_t cap, hipStream_t st,
                 std::vector<void*>& dev) {
  std::vector<size_t> off;
  size_t bytes = 0;
  for (const auto& p : parts) {
    bytes = (bytes + 255) & ~(size_t)255;
    off.push_back(bytes);
    bytes += p.second;
  }
  if (bytes + 1024 > cap) return fail(GPR_ERR_WORKSPACE, "table arena too small (%zu > %zu)", bytes + 1024, cap);
  dev.clear();
  for (size_t o : off) dev.push_back((char*)arena + o);
  if (bytes == 0) return GPR_OK;
  DevRes* R = nullptr;
  int rc = current_res(&R);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(R->mu);
  if (R->slot[R->next].cap < bytes && (rc = grow_slots(R, bytes * 2))) return rc;
  StageSlot& s = R->slot[R->next];
  R->next = (R->next + 1) % kStageSlots;
  if (!s.ev) HIPCHK(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
  if (s.inflight) HIPCHK(hipEventSynchronize(s.ev));   // the ring wrapped onto a copy still queued
  for (size_t i = 0; i < parts.size(); ++i)
    if (parts[i].second) memcpy(s.host + off[i], parts[i].first, parts[i].second);
  HIPCHK(hipMemcpyAsync(arena, s.host, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(s.ev, st));
  s.inflight = true;
  return GPR_OK;
}

// Auxiliary stream and events of the look-ahead on the current device.
int aux_resources(int nevents, hipStream_t* aux, std::vector<hipEvent_t>** evs) {
  DevRes* R = nullptr;
  int rc = current_res(&R);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(R->mu);
  if ((rc = ensure_aux(R, nevents))) return rc;
  *aux = R->aux;
  *evs = &R->events;
  return GPR_OK;
}

// Runs a program description: record pass, table upload into `arena`, execute pass.
// nevents > 0 gives the description the auxiliary stream and that many events.
template <typename F>
int run_program(F&& describe, void* arena, size_t arena_cap, hipStream_t st, int64_t* trace_wg = nullptr,
                int nevents = 0) {
  Program P;
  P.st = st;
  P.aux = st;
  if (nevents > 0) {
    int rc = aux_resources(nevents, &P.aux, &P.events);
    if (rc) return rc;
  }
  describe(P);
  const size_t nj = P.jobs.size(), ns = P.segs.size();
  const GemmJob* dj = nullptr;
  const GemmSeg* ds = nullptr;
  if (nj) {
    int rc = upload_tables(P, arena, arena_cap, st, &dj, &ds);
    if (rc) return rc;
  }
  P.reset_for_exec(dj, ds);
  describe(P);
  if (P.jobs.size() != nj || P.segs.size() != ns) return fail(GPR_ERR_HIP, "internal: record and execute passes differ");
  if (P.err != hipSuccess) return fail(GPR_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(P.err));
  if (trace_wg) *trace_wg = P.trace_wg;
  return GPR_OK;
}


// ================================================================ Cholesky
struct CholWs {
  unsigned long long* info;   // [0]: first failing pivot (atomic min), [2]: its copy for the host
  void* panel;      // copy of the panel below the diagonal tile (TRSM source)
  float* w32;       // float32 copy of the diagonal-tile inverse (mixed)
  uint16_t* planes; // hi/mid/lo bfloat16 planes of the solved panel (split modes), stride (T-1) b^2, two sets
  void* panel_t;    // transposed tiles of the solved panel, (T-1) b^2 elements, two sets
  int32_t* dag_state;   // task-graph schedule (float64): per-task counters and the control words
  int64_t dag_ntasks;

  void* arena;
  size_t arena_cap;
};

// POTRF of diagonal tile k with its inverse: the blocked loop described at describe_cholesky.
void describe_diag(Program& P, const TileLayout& L, void* K, const CholWs& w, int64_t k) {
  const int64_t b = L.b;
  double* Dk = L.diag(K, k);
  double* Wk = L.winv(K, k);
  const int64_t fill_items = ceil_div(b * b, DAG_ELEMS_PER_ITEM);
  P.op(DAG_IDENTITY, DagOp{Wk, nullptr, b, 0, 0, 0}, fill_items,
       [=](hipStream_t s) { return launch_set_identity(Wk, b, s); }, {}, {span(Wk, b * b * 8)});
  const int64_t nbk = kInnerBlock;
  for (int64_t r0 = 0; r0 < b; r0 += nbk) {
    const int64_t jb = std::min(nbk, b - r0), rb = r0 + jb, nbelow = b - rb;
    // (the first failing pivot is an atomic minimum, which needs no ordering: the task form
    // leaves the info word out of its access ranges)
    std::vector<Span> pw{span2d(Dk + r0 * b + r0, jb, jb, b, 8), span2d(Wk + r0 * b + r0, jb, jb, b, 8)};
    if (!P.dagr) pw.push_back(span(w.info, 8));
    P.op(DAG_POTRF, DagOp{Dk + r0 * b + r0, Wk + r0 * b + r0, b, jb, k * b + r0, 0}, 1,
         [=](hipStream_t s) { return launch_potrf_block(Dk + r0 * b + r0, b, Wk + r0 * b + r0, b, (int)jb, k * b + r0, w.info, s); },
         {}, pw);
    P.gemm_begin(0);
    // block row j of W: W_j[:, 0:r0] <- W_jj W_j[:, 0:r0]  (in place, column-partitioned)
    P.job(Wk + r0 * b, b, nullptr, 0, jb, r0, 1.0, 0.0, 0);
    P.seg(Wk + r0 * b + r0, b, MODE_KC, Wk + r0 * b, b, MODE_MC, jb, A_LOWER);
    // block column j of L below the block: P_j = A[rb:, r0:rb] W_jj^T  (in place, row-partitioned)
    P.job(Dk + rb * b + r0, b, nullptr, 0, nbelow, jb, 1.0, 0.0, 0);
    P.seg(Dk + rb * b + r0, b, MODE_KC, Wk + r0 * b + r0, b, MODE_KC, jb, B_LOWER);
    P.gemm_end();
    if (nbelow > 0) {
      P.gemm_begin(0);
      // W[rb:, 0:rb] -= P_j W_j[:, 0:rb]
      P.job(Wk + rb * b, b, Wk + rb * b, b, nbelow, rb, -1.0, 1.0, 0);
      P.seg(Dk + rb * b + r0, b, MODE_KC, Wk + r0 * b, b, MODE_MC, jb, 0);
      // A[rb:, rb:] -= P_j P_j^T (lower part)
      P.job(Dk + rb * b + rb, b, Dk + rb * b + rb, b, nbelow, nbelow, -1.0, 1.0, JOB_LOWER_ONLY);
      P.seg(Dk + rb * b + r0, b, MODE_KC, Dk + rb * b + r0, b, MODE_KC, jb, 0);
      P.gemm_end();
    }
  }
  P.op(DAG_ZERO_UPPER, DagOp{Dk, nullptr, b, 0, 0, 0}, fill_items,
       [=](hipStream_t s) { return launch_zero_upper(Dk, b, s); }, {}, {span(Dk, b * b * 8)});
}

// Inputs of the TRSM of panel k (block column k below the diagonal): a copy of the panel
// (the product is computed in place) and, in the mixed modes, a float32 copy of L_kk^{-1}.
void describe_panel_copy(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, int64_t k) {
  const int64_t b = L.b, T = L.T;
  if (k >= T - 1) return;
  const void* panel = L.off(K, k + 1, k);
  const size_t pbytes = (size_t)(T - k - 1) * b * b * L.esize;
  if (P.dagr && ((((uintptr_t)w.panel) | (uintptr_t)panel | pbytes) & 15)) P.dagr->ok = false;
  P.op(DAG_COPY, DagOp{w.panel, panel, (int64_t)pbytes, 0, 0, 0}, ceil_div((int64_t)pbytes, DAG_COPY_BYTES_PER_ITEM),
       [=](hipStream_t s) { return launch_copy(w.panel, panel, pbytes, s); }, {span(panel, pbytes)},
       {span(w.panel, pbytes)});
  if (is_mixed(prec)) {
    const double* Wk = L.winv(K, k);
    P.kernel([=](hipStream_t s) { return launch_convert_f64_f32(Wk, w.w32, b * b, s); }, {span(Wk, b * b * 8)},
             {span(w.w32, b * b * 4)});
  }
}

// Adds the TRSM of panel k, X = A_panel L_kk^{-T} (one job against the inverse), to the
// open launch; returns its algorithmic flops.
double add_trsm_job(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, int64_t k) {
  const int64_t b = L.b, T = L.T;
  if (k >= T - 1) return 0.0;
  const bool mixed = is_mixed(prec);
  const int64_t prow = (T - k - 1) * b;
  P.job(L.off(K, k + 1, k), b, nullptr, 0, prow, b, 1.0, 0.0, mixed ? JOB_C_F32 : 0);
  P.seg(w.panel, b, MODE_KC, mixed ? (const void*)w.w32 : (const void*)L.winv(K, k), b, MODE_KC, b, B_LOWER);
  const double bd = (double)b;
  return (double)(T - k - 1) * bd * bd * (bd + 1.0);
}

// Transposed copies of the solved panel k's tiles, buffer set k mod 2: the trailing update
// (float64, float32) and the mixed modes' diagonal-tile SYRK read both of their operands
// m-contiguous, the operand order the main loop stages fastest (measured 4-5% over
// k-contiguous operands on the float64 update).
void* panel_t_set(const TileLayout& L, const CholWs& w, int64_t k) {
  return (char*)w.panel_t + (size_t)(k & 1) * (L.T - 1) * L.b * L.b * L.esize;
}

void describe_transpose(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, int64_t k) {
  const int64_t b = L.b, T = L.T;
  if (k >= T - 1) return;
  const void* panel = L.off(K, k + 1, k);
  void* dst = panel_t_set(L, w, k);
  const int64_t count = T - k - 1;
  const int es = L.esize;
  const size_t bytes = (size_t)count * b * b * es;
  const int64_t nbt = ceil_div(b, 64);
  P.op(DAG_TRANSPOSE, DagOp{dst, panel, b, count, es, 0}, count * nbt * nbt,
       [=](hipStream_t s) { return launch_transpose_tiles(panel, dst, b, count, es, s); }, {span(panel, bytes)},
       {span(dst, bytes)});
}

// Split modes with a tile edge that is a multiple of 256: planes in the tiled layout and
// the 256 x 256 update kernel; otherwise row-major planes and 128 x 128 macro tiles.
bool bf16_tiled(const TileLayout& L) { return L.b % 256 == 0; }

// hi/mid(/lo) bfloat16 planes of the solved panel k (split modes), buffer set k mod 2.
void describe_split(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, int64_t k) {
  const int64_t b = L.b, T = L.T;
  if (!is_bf16(prec) || k >= T - 1) return;
  const int64_t pstride = (T - 1) * b * b, count = (T - k - 1) * b * b;
  const float* panel = (const float*)L.off(K, k + 1, k);
  uint16_t* pl = w.planes + (k & 1) * 3 * pstride;
  const int np = prec == GPR_BF16X6 ? 3 : 2;
  std::vector<Span> wr;
  for (int p = 0; p < np; ++p) wr.push_back(span(pl + p * pstride, count * 2));
  const bool tiled = bf16_tiled(L);
  P.kernel([=](hipStream_t s) {
    uint16_t* lo = prec == GPR_BF16X6 ? pl + 2 * pstride : nullptr;
    return tiled ? launch_split_bf16x3_tiled(panel, count, b, pl, pl + pstride, lo, s)
                 : launch_split_bf16x3(panel, count, pl, pl + pstride, lo, s);
  }, {span(panel, count * 4)}, wr);
}

// Trailing update of step k restricted to block columns [n0, n1) (SYRK on diagonal tiles,
// GEMM elsewhere).  Mixed modes: the SYRK on the float64 diagonal tiles multiplies the
// float32 panel in float64 (exact products, so the pivots do not inherit float32
// accumulation error); the GEMM tiles use the mode's products.
// Which tiles of the block columns an update covers: the diagonal tiles (SYRK), the tiles
// below them (GEMM), or both.
enum { UPD_DIAG = 1, UPD_BELOW = 2, UPD_ALL = 3 };

void describe_update(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, int64_t k, int64_t n0,
                     int64_t n1, int part = UPD_ALL) {
  const int64_t b = L.b, T = L.T;
  if (n0 >= n1) return;
  const bool mixed = is_mixed(prec), split = is_bf16(prec);
  const int64_t pstride = (T - 1) * b * b;
  const uint16_t* pl = split ? w.planes + (k & 1) * 3 * pstride : nullptr;
  const char* pt = split ? nullptr : (const char*)panel_t_set(L, w, k);
  auto opnd = [&](int64_t m) -> const void* {
    return split ? (const void*)(pl + (m - k - 1) * b * b) : (const void*)(pt + (size_t)(m - k - 1) * b * b * L.esize);
  };
  const int mode = split ? MODE_KC : MODE_MC;   // transposed panel tiles: element (r, c) at [c b + r]
  const double bd = (double)b;
  double syrk_flops = 0.0, gemm_flops = 0.0;
  for (int64_t nn = n0; nn < n1; ++nn) {
    if (part & UPD_DIAG) syrk_flops += bd * bd * (bd + 1.0);
    if (part & UPD_BELOW) gemm_flops += 2.0 * (double)(T - nn - 1) * bd * bd * bd;
  }
  if (mixed && (part & UPD_DIAG)) {
    // the SYRK into the float64 diagonal tiles, float64 products of the float32 panel,
    // both operands m-contiguous from the transposed panel tiles
    const char* ptk = (const char*)panel_t_set(L, w, k);
    P.gemm_begin(0, GEMM_KIND_WIDEN);
    for (int64_t m = n0; m < n1; ++m) {
      double* Cm = L.diag(K, m);
      const void* Tm = ptk + (size_t)(m - k - 1) * b * b * L.esize;
      P.job(Cm, b, Cm, b, b, b, -1.0, 1.0, JOB_LOWER_ONLY);
      P.seg(Tm, b, MODE_MC, Tm, b, MODE_MC, b, 0);
    }
    P.gemm_end();
  }
  const bool t256 = split && bf16_tiled(L);
  const int kind = !split ? GEMM_KIND_UPDATE
                          : (prec == GPR_BF16X6 ? (t256 ? GEMM_KIND_BF16X6_T256 : GEMM_KIND_BF16X6)
                                                : (t256 ? GEMM_KIND_BF16X3_T256 : GEMM_KIND_BF16X3));
  P.gemm_begin(mixed, kind, mixed ? gemm_flops : syrk_flops + gemm_flops);
  for (int64_t nn = n0; nn < n1; ++nn) {
    for (int64_t m = nn; m < T; ++m) {
      if (m == nn) {
        if (mixed || !(part & UPD_DIAG)) continue;
        double* Cm = L.diag(K, m);
        P.job(Cm, b, Cm, b, b, b, -1.0, 1.0, JOB_LOWER_ONLY);
      } else {
        if (!(part & UPD_BELOW)) continue;
        void* Cmn = L.off(K, m, nn);
        P.job(Cmn, b, Cmn, b, b, b, -1.0, 1.0, mixed ? JOB_C_F32 : 0);
      }
      P.seg(opnd(m), b, mode, opnd(nn), b, mode, b, 0);
      if (split) P.segs.back().pstrideA = P.segs.back().pstrideB = pstride;
    }
  }
  P.gemm_end();
}

// The tiled right-looking factorisation (Fig. 1).  Step k: factor the diagonal tile
// and invert its factor (POTRF), X_mk = A_mk L_kk^{-T} for the panel (TRSM, one GEMM
// against the inverse), then A_mn -= X_mk X_nk^T over the trailing lower triangle
// (SYRK on diagonal tiles, GEMM elsewhere) as batched launches.  Without the look-ahead
// all of it goes to the caller's stream in that order, one update launch per step.
//
// Look-ahead (default): each step's update is issued as block column k+1 (U1) and the
// remaining columns (U2), in the mixed modes with diagonal tile k+1 first on its own (U0).
// The factorisation of diagonal tile k+1 runs on the auxiliary stream as soon as U1 (mixed:
// U0, beside U1) is done, and the solve of its panel once U1 is done, overlapping U2 on
// the caller's stream; events order the two (e0(k): U0 of step k done, e1(k): U1 done,
// e2(k): panel k solved).  The
// two streams touch disjoint tiles: U2 reads block column k and writes columns >= k+2,
// the look-ahead work reads and writes block column k+1, diagonal tile k+1 and its
// inverse, the panel copy and the operands of the next update built from panel k+1 (its
// transposed tiles, or in the split modes its bfloat16 planes), which are double-buffered
// by step parity.  The panel is staged by a copy kernel: a runtime
// device-to-device copy issued on the auxiliary stream read stale panel data produced by
// U1 on the other stream (run-to-run differences of 1e-5 in the solve residual at
// n = 65536), which the copy kernel does not.
//
// The diagonal tile itself is factored by a blocked right-looking loop with blocks of
// 64; its inverse W is accumulated in the same loop: starting from W = I, block
// step j multiplies block row j of W by the block inverse W_jj and subtracts
// P_j (W_jj W_j) from the rows below, P_j being the block column of L below the
// diagonal block; that update shares its launch with the trailing update P_j P_j^T.
int chol_events_needed(int64_t T) { return 1 + 3 * (int)T; }

// Schedule of the factorisation (gpr_set_schedule): GPR_SCHEDULE_STREAM (every launch on the
// caller's stream), GPR_SCHEDULE_LOOKAHEAD (two streams, the default) or GPR_SCHEDULE_DEVICE
// (the task graph executed by a persistent kernel; float64 only, other precisions use the
// look-ahead).  All give the same bits.
std::atomic<int> g_schedule{GPR_SCHEDULE_LOOKAHEAD};

void describe_cholesky(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w, bool lookahead) {
  const int64_t T = L.T;
  auto panel = [&](int64_t k) {
    describe_panel_copy(P, L, K, prec, w, k);
    if (k < T - 1) {
      P.gemm_begin(is_mixed(prec));
      add_trsm_job(P, L, K, prec, w, k);
      P.gemm_end();
    }
    describe_transpose(P, L, K, prec, w, k);
    describe_split(P, L, K, prec, w, k);
  };
  auto diag_and_panel = [&](int64_t k) {
    describe_diag(P, L, K, w, k);
    panel(k);
  };
  auto e0 = [](int64_t k) { return 1 + 3 * (int)k; };   // step k's update of diagonal tile k+1 done
  auto e1 = [](int64_t k) { return 2 + 3 * (int)k; };   // step k's update of block column k+1 done
  auto e2 = [](int64_t k) { return 3 + 3 * (int)k; };   // panel k solved
  unsigned long long* info = w.info;
  P.on(0);
  P.kernel([=](hipStream_t s) { return launch_fill_u64(info, ~0ull, 2, s); }, {}, {span(info, 16)});
  if (!lookahead) {
    // one stream: step k's diagonal tile, panel, then its whole trailing update (one launch)
    for (int64_t k = 0; k < T; ++k) {
      diag_and_panel(k);
      describe_update(P, L, K, prec, w, k, k + 1, T);
    }
    P.kernel([=](hipStream_t s) { return launch_copy(info + 2, info, 2 * sizeof(unsigned long long), s); },
             {span(info, 16)}, {span(info + 2, 16)});
    return;
  }
  P.record(0);
  P.on(1);
  P.wait(0);
  diag_and_panel(0);
  P.record(e2(0));
  // The mixed modes update the float64 diagonal tiles in a launch of their own (U0), so the
  // factorisation of diagonal tile k+1 can start beside U1.  In float64 the diagonal tile's
  // SYRK shares U1's launch: on its own it would fill only half the GPU (its lower
  // macro tiles), which costs about what the overlap gains.
  const bool split_u0 = is_mixed(prec);
  for (int64_t k = 0; k + 1 < T; ++k) {
    P.on(0);
    P.wait(e2(k));
    if (split_u0) {
      describe_update(P, L, K, prec, w, k, k + 1, k + 2, UPD_DIAG);    // U0: diagonal tile k+1
      P.record(e0(k));
      describe_update(P, L, K, prec, w, k, k + 1, k + 2, UPD_BELOW);   // U1: the rest of block column k+1
    } else {
      describe_update(P, L, K, prec, w, k, k + 1, k + 2);              // U1: block column k+1
    }
    P.record(e1(k));
    describe_update(P, L, K, prec, w, k, k + 2, T);                    // U2: the remaining columns
    P.on(1);
    if (split_u0) {
      P.wait(e0(k));
      describe_diag(P, L, K, w, k + 1);   // beside U1: it reads only diagonal tile k+1
      P.wait(e1(k));
    } else {
      P.wait(e1(k));
      describe_diag(P, L, K, w, k + 1);
    }
    panel(k + 1);
    P.record(e2(k + 1));
  }
  P.on(0);
  P.wait(e2(T - 1));
  // the first failing pivot (written by atomics on the auxiliary stream), copied by a kernel
  // on the caller's stream into the slot the host reads
  P.kernel([=](hipStream_t s) { return launch_copy(info + 2, info, 2 * sizeof(unsigned long long), s); },
           {span(info, 16)}, {span(info + 2, 16)});
}

// The factorisation as a task graph: the one-stream order of describe_cholesky with the
// trailing update of each step split into one task per block column, so that the
// dependencies, not the issue order, decide what overlaps (the next diagonal tile may
// start once its own column is updated, any later column's update once its inputs are
// ready).  The pivot word is reset before and copied after the graph, on the stream.
void describe_cholesky_graph(Program& P, const TileLayout& L, void* K, int prec, const CholWs& w) {
  const int64_t T = L.T;
  for (int64_t k = 0; k < T; ++k) {
    // the critical path -- diagonal tile, panel, the next block column's update -- is
    // served first from the first ready queue
    if (P.dagr) P.dagr->prio = 0;
    describe_diag(P, L, K, w, k);
    describe_panel_copy(P, L, K, prec, w, k);
    if (k < T - 1) {
      P.gemm_begin(is_mixed(prec));
      add_trsm_job(P, L, K, prec, w, k);
      P.gemm_end();
    }
    describe_transpose(P, L, K, prec, w, k);
    describe_split(P, L, K, prec, w, k);
    for (int64_t c = k + 1; c < T; ++c) {
      if (P.dagr) P.dagr->prio = c == k + 1 ? 0 : 1;
      describe_update(P, L, K, prec, w, k, c, c + 1);
    }
  }
}

// Successor lists of a recorded graph.  Task u precedes task t (u issued first) when t
// reads what u writes, writes what u reads or writes what u writes, at a granularity of
// 1 MiB (coarser ranges only add edges).  Returns false when the edges exceed `max_succ`.
constexpr int kDagGranuleShift = 20;

bool dag_edges(DagRecord& R, std::vector<int32_t>& succ, size_t max_succ) {
  struct Gran {
    int32_t writer = -1;
    std::vector<int32_t> readers;
  };
  const int nt = (int)R.tasks.size();
  std::unordered_map<uint64_t, Gran> g;
  g.reserve(1 << 16);
  std::vector<std::vector<int32_t>> preds(nt);
  std::vector<int32_t> stamp(nt, -1);
  for (int t = 0; t < nt; ++t) {
    auto add = [&](int32_t u) {
      if (u >= 0 && u != t && stamp[u] != t) {
        stamp[u] = t;
        preds[t].push_back(u);
      }
    };
    for (const Span& sp : R.rd[t]) {
      if (sp.hi <= sp.lo) continue;
      for (uint64_t q = sp.lo >> kDagGranuleShift; q <= (sp.hi - 1) >> kDagGranuleShift; ++q) {
        Gran& e = g[q];
        add(e.writer);
        if (e.readers.empty() || e.readers.back() != t) e.readers.push_back(t);
      }
    }
    for (const Span& sp : R.wr[t]) {
      if (sp.hi <= sp.lo) continue;
      for (uint64_t q = sp.lo >> kDagGranuleShift; q <= (sp.hi - 1) >> kDagGranuleShift; ++q) {
        Gran& e = g[q];
        add(e.writer);
        for (int32_t r : e.readers) add(r);
        e.writer = t;
        e.readers.clear();
      }
    }
  }
  std::vector<int32_t> nsucc(nt, 0);
  size_t edges = 0;
  for (int t = 0; t < nt; ++t) {
    R.tasks[t].npred = (int32_t)preds[t].size();
    for (int32_t u : preds[t]) ++nsucc[u];
    edges += preds[t].size();
  }
  if (edges > max_succ) return false;
  int32_t off = 0;
  for (int t = 0; t < nt; ++t) {
    R.tasks[t].succ0 = off;
    R.tasks[t].nsucc = 0;
    off += nsucc[t];
  }
  succ.assign(edges, 0);
  for (int t = 0; t < nt; ++t)
    for (int32_t u : preds[t]) succ[R.tasks[u].succ0 + R.tasks[u].nsucc++] = t;
  return true;
}

// Table bytes of a graph with nt tasks, ns successor entries and no ops, beyond the jobs.
size_t dag_max_succ(size_t ntasks) { return 16 * ntasks + 1024; }
size_t dag_table_bytes(const Program& P, const DagRecord& R) {
  auto r256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return r256(P.jobs.size() * sizeof(GemmJob)) + r256(P.segs.size() * sizeof(GemmSeg)) +
         r256(R.tasks.size() * sizeof(DagTask)) + r256(dag_max_succ(R.tasks.size()) * sizeof(int32_t)) +
         r256(R.ops.size() * sizeof(DagOp)) + 1024;
}

// Number of tasks of the float64 graph of a layout (recorded once per (n, b), then cached).
CholWs carve_chol(void* ws, const TileLayout& L, int prec, size_t ws_bytes, bool with_dag = true);

int64_t dag_task_count(const TileLayout& L) {
  static std::mutex mu;
  static std::map<std::pair<int64_t, int64_t>, int64_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({L.n, L.b});
  if (it != cache.end()) return it->second;
  Program P;
  DagRecord R;
  P.dagr = &R;
  const CholWs w = carve_chol(kSymWs, L, GPR_FP64, 0, false);
  describe_cholesky_graph(P, L, kSymK, GPR_FP64, w);
  const int64_t nt = (int64_t)R.tasks.size();
  cache[{L.n, L.b}] = nt;
  return nt;
}

struct CholSizes {
  size_t fixed, arena;
};

CholSizes chol_sizes(const TileLayout& L, int prec) {
  Carve c(nullptr);
  c.take<char>(256);
  c.take<char>((size_t)(L.T > 1 ? L.T - 1 : 0) * L.b * L.b * L.esize);
  if (is_mixed(prec)) c.take<float>((size_t)L.b * L.b);
  if (is_bf16(prec)) c.take<uint16_t>((size_t)6 * (L.T > 1 ? L.T - 1 : 0) * L.b * L.b);
  c.take<char>((size_t)2 * (L.T > 1 ? L.T - 1 : 0) * L.b * L.b * L.esize);
  Program P1, P2;
  const CholWs w = carve_chol(kSymWs, L, prec, 0, false);
  describe_cholesky(P1, L, kSymK, prec, w, false);
  describe_cholesky(P2, L, kSymK, prec, w, true);
  size_t arena = std::max(arena_bytes_of(P1), arena_bytes_of(P2));
  if (prec == GPR_FP64) {
    // the task graph's tables and its per-task counters
    Program P3;
    DagRecord R;
    P3.dagr = &R;
    describe_cholesky_graph(P3, L, kSymK, prec, w);
    arena = std::max(arena, dag_table_bytes(P3, R));
    c.take<int32_t>(dag_state_ints(dag_task_count(L)));
  }
  return CholSizes{c.off, arena};
}

CholWs carve_chol(void* ws, const TileLayout& L, int prec, size_t ws_bytes, bool with_dag) {
  Carve c(ws);
  CholWs w{};
  w.info = c.take<unsigned long long>(32);
  w.panel = c.take<char>((size_t)(L.T > 1 ? L.T - 1 : 0) * L.b * L.b * L.esize);
  w.w32 = is_mixed(prec) ? c.take<float>((size_t)L.b * L.b) : nullptr;
  w.planes = is_bf16(prec) ? c.take<uint16_t>((size_t)6 * (L.T > 1 ? L.T - 1 : 0) * L.b * L.b) : nullptr;
  w.panel_t = c.take<char>((size_t)2 * (L.T > 1 ? L.T - 1 : 0) * L.b * L.b * L.esize);
  if (prec == GPR_FP64 && with_dag) {
    w.dag_ntasks = dag_task_count(L);
    w.dag_state = c.take<int32_t>(dag_state_ints(w.dag_ntasks));
  }
  w.arena = c.take<char>(0);
  w.arena_cap = ws_bytes > c.off ? ws_bytes - c.off : 0;
  return w;
}

// ================================================================ triangular solves
struct SolveWs {
  double *r, *z, *t, *partial, *kpart, *kcol, *res, *dvec;
  double* xp;   // padded solution (T b) when the tile does not divide n
};

size_t solve_partial_rows(const TileLayout& L) {
  const int64_t rows = std::max<int64_t>((L.T - 1) * L.b, L.b);
  return (size_t)ceil_div(std::max<int64_t>(rows, 1), kRowsPerChunk);
}

SolveWs carve_solve(Carve& c, const TileLayout& L) {
  SolveWs w{};
  const int64_t n = L.n, b = L.b, npad = L.npad();
  w.r = c.take<double>(npad);
  w.z = c.take<double>(npad);
  w.t = c.take<double>(b);
  w.partial = c.take<double>(solve_partial_rows(L) * b);
  // partial sums of the residual's K alpha: per chunk of kColsPerChunk points (Matern), or
  // per 128-point block column (kpart) and block row (kcol) of the symmetric products
  w.kpart = c.take<double>((size_t)ceil_div(std::max<int64_t>(n, 1), std::min<int64_t>(kColsPerChunk, GEMM_BM)) * n);
  w.kcol = c.take<double>((size_t)ceil_div(std::max<int64_t>(n, 1), GEMM_BM) * n);
  w.res = c.take<double>(n);
  w.dvec = c.take<double>(n);
  w.xp = npad > n ? c.take<double>(npad) : nullptr;
  return w;
}

// x = (L L^T)^{-1} y with L in tiles; the diagonal-tile inverses turn every step into a
// matrix-vector product.  Forward: z_j = W_jj r_j, then r_below -= L_(below,j) z_j.
// Backward: t = z_i - L_(below,i)^T x_below, then x_i = W_ii^T t.
// y and x have n entries; the substitutions run on T b entries, the right-hand side padded
// with zeros (the padded solution is zero too and is dropped).
int tri_solve(const TileLayout& L, const void* K, const double* yin, double* xout, const SolveWs& w,
              hipStream_t st) {
  const int64_t b = L.b, T = L.T, n = L.n, npad = L.npad();
  const int f32 = L.esize == 4;
  void* Kc = const_cast<void*>(K);
  double* x = npad > n ? w.xp : xout;
  HIPCHK(launch_copy(w.r, yin, n * sizeof(double), st));
  if (npad > n) HIPCHK(launch_fill_u64((unsigned long long*)(w.r + n), 0ull, npad - n, st));
  for (int64_t j = 0; j < T; ++j) {
    HIPCHK(launch_gemv_n(L.winv(Kc, j), 0, b, b, b, w.r + j * b, 1.0, nullptr, 0.0, w.z + j * b, st));
    if (j < T - 1) {
      const int64_t rows = (T - j - 1) * b;
      HIPCHK(launch_gemv_n(L.off(Kc, j + 1, j), f32, b, rows, b, w.z + j * b, -1.0, w.r + (j + 1) * b, 1.0,
                           w.r + (j + 1) * b, st));
    }
  }
  const int64_t nchb = ceil_div(b, kRowsPerChunk);
  for (int64_t i = T - 1; i >= 0; --i) {
    const double* t = w.z + i * b;
    if (i < T - 1) {
      const int64_t rows = (T - i - 1) * b;
      HIPCHK(launch_gemv_t_partial(L.off(Kc, i + 1, i), f32, b, rows, b, x + (i + 1) * b, w.partial, kRowsPerChunk, st));
      HIPCHK(launch_reduce_partials(w.partial, ceil_div(rows, kRowsPerChunk), b, -1.0, w.z + i * b, 1.0, w.t, st));
      t = w.t;
    }
    HIPCHK(launch_gemv_t_partial(L.winv(Kc, i), 0, b, b, b, t, w.partial, kRowsPerChunk, st));
    HIPCHK(launch_reduce_partials(w.partial, nchb, b, 1.0, nullptr, 0.0, x + i * b, st));
  }
  if (x != xout) HIPCHK(launch_copy(xout, x, n * sizeof(double), st));
  return GPR_OK;
}

int solve_impl(const TileLayout& L, const void* K, const double* Z, int64_t d, HyperArg h, const double* y,
               double* alpha, int sweeps, const SolveWs& w, hipStream_t st) {
  int rc = tri_solve(L, K, y, alpha, w, st);
  if (rc) return rc;
  const int64_t n = L.n;
  for (int s = 0; s < sweeps; ++s) {
    // r = y - K alpha in float64, K regenerated from Z (matrix-free)
    if (h.kernel == KERNEL_SE) {
      // the symmetry of K halves the pairs
      HIPCHK(launch_se_kmatvec_gram_sym(Z, n, d, h, alpha, w.kpart, w.kcol, st));
      HIPCHK(launch_residual_finish_sym(w.kpart, w.kcol, n, h, y, alpha, w.res, st));
    } else {
      HIPCHK(launch_kmatvec_partial(Z, n, Z, n, d, h, alpha, w.kpart, kColsPerChunk, st));
      HIPCHK(launch_residual_finish(w.kpart, ceil_div(n, kColsPerChunk), n, h, y, alpha, w.res, st));
    }
    rc = tri_solve(L, K, w.res, w.dvec, w, st);
    if (rc) return rc;
    HIPCHK(launch_axpy(alpha, w.dvec, 1.0, n, st));
  }
  return GPR_OK;
}

// ================================================================ variance
struct VarWs {
  void* V;         // T b x m (float64, or float32 in mixed modes); rows n.. are zero
  void* tmp;       // b x m
  void* rowt;      // block row i of L with each tile transposed: (T-1) b x b tiles
  float* w32;      // T b x b float32 copies of the diagonal-tile inverses (mixed)
  double* partial; // column sums of squares
  // split modes (tiles and m multiples of 256): bfloat16 planes of the products' operands,
  // plane strides *s elements: V_j^T for every block j (m x b each), block row i of L and
  // W_ii (T tiles), the right-hand side of W_ii (m x b)
  uint16_t *pv, *pl, *pt;
  int64_t pvs, pls, pts;
  void* arena;
};

// The split modes run the variance's forward substitution from bfloat16 planes when the
// tiles and the number of test points suit the 256 x 256 kernels, float32 otherwise.
bool var_split(const TileLayout& L, int64_t m, int prec) {
  return is_bf16(prec) && bf16_tiled(L) && m > 0 && m % 256 == 0;
}

void describe_var(Program& P, const TileLayout& L, const void* Kc, int64_t m, int prec, const VarWs& w) {
  const int64_t b = L.b, T = L.T;
  const bool mixed = is_mixed(prec);
  void* K = const_cast<void*>(Kc);
  const int es = mixed ? 4 : 8;
  const int cflag = mixed ? JOB_C_F32 : 0;
  for (int64_t i = 0; i < T; ++i) {
    char* Vi = (char*)w.V + (size_t)i * b * m * es;
    // tmp = B_i - sum_{j<i} L_ij V_j, with the tiles L_ij transposed first so that both
    // operands are m-contiguous
    if (i > 0) {
      const void* obase = L.off(K, 1, 0);   // region O
      void* rowt = w.rowt;
      const int64_t Tt = T, bi = b;
      P.kernel([=](hipStream_t s) { return launch_transpose_block_row(obase, Tt, i, rowt, bi, es, s); });
    }
    P.gemm_begin(mixed);
    P.job(w.tmp, m, Vi, m, b, m, -1.0, 1.0, cflag);
    for (int64_t j = 0; j < i; ++j)
      P.seg((char*)w.rowt + (size_t)j * b * b * es, b, MODE_MC, (char*)w.V + (size_t)j * b * m * es, m, MODE_MC, b, 0);
    P.gemm_end();
    // V_i = W_ii tmp
    P.gemm_begin(mixed);
    P.job(Vi, m, nullptr, 0, b, m, 1.0, 0.0, cflag);
    P.seg(mixed ? (const void*)(w.w32 + (size_t)i * b * b) : (const void*)L.winv(K, i), b, MODE_KC, w.tmp, m,
          MODE_MC, b, A_LOWER);
    P.gemm_end();
  }
}

// describe_var from split-bfloat16 planes (var_split): block i splits L_ij (j < i) as
// stored, then tmp = B_i - sum_j L_ij V_j against the planes of V_j^T kept from earlier
// blocks; then it splits W_ii and the right-hand side transposed, V_i = W_ii tmp (W_ii in
// full, with its zeros), and keeps the planes of V_i^T for the later blocks.  V stays
// float32 for the float64 sums of squares and the full covariance.
void describe_var_split(Program& P, const TileLayout& L, const void* Kc, int64_t m, int prec, const VarWs& w) {
  const int64_t b = L.b, T = L.T, bb = b * b;
  const int np = prec == GPR_BF16X6 ? 3 : 2;
  const int kind = prec == GPR_BF16X6 ? GEMM_KIND_BF16X6_SOLVE_T256 : GEMM_KIND_BF16X3_SOLVE_T256;
  void* K = const_cast<void*>(Kc);
  auto split = [&](std::vector<const float*> src, int64_t rows, int64_t ld, bool trans, uint16_t* out, int64_t ps) {
    P.kernel([=](hipStream_t s) {
      return launch_split_bf16_tiles(src.data(), (int64_t)src.size(), rows, b, ld, trans, out, ps, np, s);
    });
  };
  float* const V = (float*)w.V;
  float* const tmp = (float*)w.tmp;
  uint16_t* const wslot = w.pl + (T - 1) * bb;   // W_ii (block row i of L uses slots 0 .. i-1)
  for (int64_t i = 0; i < T; ++i) {
    float* Vi = V + i * b * m;
    const float* rhs = Vi;
    if (i > 0) {
      std::vector<const float*> row(i);
      for (int64_t j = 0; j < i; ++j) row[j] = (const float*)L.off(K, i, j);
      split(row, b, b, false, w.pl, w.pls);
      P.gemm_begin(1, kind);
      P.job(tmp, m, Vi, m, b, m, -1.0, 1.0, JOB_C_F32);
      for (int64_t j = 0; j < i; ++j) {
        P.seg(w.pl + j * bb, b, MODE_KC, w.pv + j * b * m, b, MODE_KC, b, 0);
        P.segs.back().pstrideA = w.pls;
        P.segs.back().pstrideB = w.pvs;
      }
      P.gemm_end();
      rhs = tmp;
    }
    split({rhs}, m, m, true, w.pt, w.pts);
    split({w.w32 + i * bb}, b, b, false, wslot, w.pls);
    P.gemm_begin(1, kind);
    P.job(Vi, m, nullptr, 0, b, m, 1.0, 0.0, JOB_C_F32);
    P.seg(wslot, b, MODE_KC, w.pt, b, MODE_KC, b, 0);
    P.segs.back().pstrideA = w.pls;
    P.segs.back().pstrideB = w.pts;
    P.gemm_end();
    if (i < T - 1) split({Vi}, m, m, true, w.pv + i * b * m, w.pvs);
  }
}

void describe_variance(Program& P, const TileLayout& L, const void* Kc, int64_t m, int prec, const VarWs& w) {
  if (var_split(L, m, prec)) describe_var_split(P, L, Kc, m, prec, w);
  else describe_var(P, L, Kc, m, prec, w);
}

// Sigma = K_{Zs,Zs} - V^T V: float64 products and accumulation in every precision (the
// mixed modes store V in float32 and widen each product to float64).
void describe_fullcov(Program& P, const TileLayout& L, int64_t m, int prec, const VarWs& w, double* out) {
  const bool mixed = is_mixed(prec);
  P.gemm_begin(0, mixed ? GEMM_KIND_WIDEN : GEMM_KIND_GENERIC);
  P.job(out, m, out, m, m, m, -1.0, 1.0, 0);
  P.seg(w.V, m, MODE_MC, w.V, m, MODE_MC, L.npad(), 0);
  P.gemm_end();
}

VarWs carve_var(Carve& c, const TileLayout& L, int64_t m, int prec) {
  VarWs w{};
  const int es = is_mixed(prec) ? 4 : 8;
  w.V = c.take<char>((size_t)L.npad() * m * es);
  w.tmp = c.take<char>((size_t)L.b * m * es);
  const bool split = var_split(L, m, prec);
  w.rowt = split ? nullptr : c.take<char>((size_t)(L.T > 1 ? L.T - 1 : 0) * L.b * L.b * es);
  w.w32 = is_mixed(prec) ? c.take<float>((size_t)L.T * L.b * L.b) : nullptr;
  w.partial = c.take<double>((size_t)ceil_div(std::max<int64_t>(L.n, 1), kRowsPerChunk) * m);
  if (split) {
    const int np = prec == GPR_BF16X6 ? 3 : 2;
    w.pvs = L.npad() * m;
    w.pls = L.T * L.b * L.b;
    w.pts = m * L.b;
    w.pv = c.take<uint16_t>((size_t)np * w.pvs);
    w.pl = c.take<uint16_t>((size_t)np * w.pls);
    w.pt = c.take<uint16_t>((size_t)np * w.pts);
  }
  w.arena = c.take<char>(0);
  return w;
}

// ================================================================ gradient
struct GradWs {
  void* panel;      // block column of L with each tile transposed: (T-1) b x b tiles
  void* row;        // copy of one block row of the residual: (T-1) b x b tiles
  float* w32;       // T b x b (mixed)
  uint16_t* pa;     // split modes, tiles a multiple of 256: bfloat16 planes of T tiles each
  uint16_t* pb;     //   (A and B operands of the products), plane stride pstride elements
  int64_t pstride;
  double* partial;  // [trace workgroups][3]
  int64_t partial_wg;
  double* u;        // r^2 / (2 l^2) of every lower tile pair: T (T+1) / 2 float64 tiles
  double* apad;     // alpha padded with zeros to T b (when the tile does not divide n)
  void* arena;
};

// Number of workgroups of all gradient-trace launches (one per macro tile of every job).
int64_t trace_workgroups(const TileLayout& L) {
  const int64_t tpt = ceil_div(L.b, GEMM_BM) * ceil_div(L.b, GEMM_BN);
  return L.T * (L.T + 1) * (L.T + 2) / 6 * tpt;
}

// X = L^{-1} in place over region O, right-looking in the order of forward substitution
// (X_jj = L_jj^{-1} is region W).  R holds the running right-hand side of L X = I; step j
//   finalises block row j:     X_jc = L_jj^{-1} R_jc                  (c < j)
//   eliminates block column j: R_ic -= L_ij X_jc (c < j), R_ij = -L_ij L_jj^{-1}  (i > j)
// Each step is one launch of single-segment tile products sharing block row j and the
// transposed copy of block column j, so concurrently running workgroups reuse the same operands.
void describe_trtri(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  const int64_t b = L.b, T = L.T;
  const bool mixed = is_mixed(prec);
  const size_t tb = (size_t)b * b * (mixed ? 4 : 8);
  const int cflag = mixed ? JOB_C_F32 : 0;
  const double bd = (double)b, trmm = bd * bd * (bd + 1.0), gemm = 2.0 * bd * bd * bd;
  auto Wd = [&](int64_t i) -> const void* {
    return mixed ? (const void*)(w.w32 + (size_t)i * b * b) : (const void*)L.winv(K, i);
  };
  for (int64_t j = 0; j < T; ++j) {
    if (j > 0) {
      for (int64_t c = 0; c < j; ++c) {
        void* dst = (char*)w.row + c * tb;
        const void* src = L.off(K, j, c);
        P.kernel([=](hipStream_t s) { return launch_copy(dst, src, tb, s); });
      }
      P.gemm_begin(mixed, GEMM_KIND_TRTRI, (double)j * trmm);
      for (int64_t c = 0; c < j; ++c) {
        P.job(L.off(K, j, c), b, nullptr, 0, b, b, 1.0, 0.0, cflag);
        P.seg(Wd(j), b, MODE_KC, (char*)w.row + c * tb, b, MODE_MC, b, A_LOWER);
      }
      P.gemm_end();
    }
    if (j == T - 1) break;
    // block column j of L, transposed tile by tile: both operands of the elimination are
    // then m-contiguous, the operand order the main loop stages fastest
    const void* col = L.off(K, j + 1, j);
    const int64_t ncol = T - j - 1;
    const int es = mixed ? 4 : 8;
    P.kernel([=](hipStream_t s) { return launch_transpose_tiles(col, w.panel, b, ncol, es, s); });
    P.gemm_begin(mixed, GEMM_KIND_TRTRI, (double)(T - j - 1) * ((double)j * gemm + trmm));
    for (int64_t i = j + 1; i < T; ++i) {
      const void* Pi = (const char*)w.panel + (i - j - 1) * tb;
      for (int64_t c = 0; c < j; ++c) {
        void* C = L.off(K, i, c);
        P.job(C, b, C, b, b, b, -1.0, 1.0, cflag);
        P.seg(Pi, b, MODE_MC, L.off(K, j, c), b, MODE_MC, b, 0);
      }
      P.job(L.off(K, i, j), b, nullptr, 0, b, b, -1.0, 0.0, cflag);
      P.seg(Pi, b, MODE_MC, Wd(j), b, MODE_MC, b, B_UPPER);
    }
    P.gemm_end();
  }
}

// K^{-1} = sum_k X_k^T X_k over the block rows X_k of X = L^{-1}: step k adds X_ki^T X_kj
// to every lower tile pair j <= i <= k, and the trace epilogue contracts that contribution
// with the gradient weights at once, so no K^{-1} tile is stored; alpha alpha^T is
// subtracted once per tile pair, in the step k = i.  One launch per k, all of whose jobs
// share block row k.  Diagonal tile pairs (i = j) are symmetric: only their macro tiles on
// and below the diagonal run (the epilogue doubles the strictly-lower entries), so the
// flops of all launches add up to those of the LAUUM product, about n^3 / 3.
void describe_lauum_trace(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  const int64_t b = L.b, T = L.T;
  const bool mixed = is_mixed(prec);
  const double bd = (double)b;
  // a full tile product, a lower half of a symmetric or a triangular-times-full one, the
  // lower half of a product of two triangular tiles
  const double full = 2.0 * bd * bd * bd, half = bd * bd * (bd + 1.0), tri3 = bd * (bd + 1.0) * (bd + 2.0) / 3.0;
  auto Wd = [&](int64_t i) -> const void* {
    return mixed ? (const void*)(w.w32 + (size_t)i * b * b) : (const void*)L.winv(K, i);
  };
  for (int64_t k = 0; k < T; ++k) {
    const double kd = (double)k;
    P.gemm_begin(mixed, GEMM_KIND_TRACE, kd * (kd - 1.0) / 2.0 * full + 2.0 * kd * half + tri3);
    for (int64_t i = 0; i <= k; ++i) {
      const void* A = (i == k) ? Wd(k) : L.off(K, k, i);
      for (int64_t j = 0; j <= i; ++j) {
        const void* Bp = (j == k) ? Wd(k) : L.off(K, k, j);
        int tri = 0;
        if (i == k) tri |= A_UPPER;
        if (j == k) tri |= B_UPPER;
        const int flags = (i == k ? JOB_TRACE_ALPHA : 0) | (i == j ? JOB_LOWER_ONLY : 0);
        P.job(nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, flags, (int)i, (int)j);
        P.seg(A, b, MODE_MC, Bp, b, MODE_MC, b, tri);
      }
    }
    P.gemm_end();
  }
}

// The inversion of describe_trtri from split-bfloat16 planes (tiles a multiple of 256):
// before each launch the operand tiles are split into planes in the tiled layout, the A
// operands as stored, the B operands transposed (the kernels take C = A B^T with both
// operands k-contiguous), and the triangular tiles W_jj as full tiles with their zeros.
// The planes are copies, so the products may overwrite their sources: step j splits
//   W_jj and R_jc^T (c < j), then X_jc = W_jj R_jc in place;
//   L_ij (i > j), X_jc^T and W_jj^T, then R_ic -= L_ij X_jc and R_ij = -L_ij W_jj in place.
void describe_trtri_split(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  const int64_t b = L.b, T = L.T, bb = b * b, ps = w.pstride;
  const int np = prec == GPR_BF16X6 ? 3 : 2;
  const int kind = prec == GPR_BF16X6 ? GEMM_KIND_BF16X6_TRTRI_T256 : GEMM_KIND_BF16X3_TRTRI_T256;
  const double bd = (double)b, trmm = bd * bd * (bd + 1.0), gemm = 2.0 * bd * bd * bd;
  uint16_t* const pa = w.pa;
  uint16_t* const pb = w.pb;
  auto split = [&](std::vector<const float*> src, bool trans, uint16_t* out) {
    P.kernel([=](hipStream_t s) {
      return launch_split_bf16_tiles(src.data(), (int64_t)src.size(), b, b, b, trans, out, ps, np, s);
    });
  };
  auto seg = [&](const uint16_t* A, const uint16_t* B) {
    P.seg(A, b, MODE_KC, B, b, MODE_KC, b, 0);
    P.segs.back().pstrideA = P.segs.back().pstrideB = ps;
  };
  for (int64_t j = 0; j < T; ++j) {
    const float* Wj = w.w32 + j * bb;
    if (j > 0) {
      std::vector<const float*> r(j);
      for (int64_t c = 0; c < j; ++c) r[c] = (const float*)L.off(K, j, c);
      split(r, true, pb);
      split({Wj}, false, pa);
      P.gemm_begin(1, kind, (double)j * trmm);
      for (int64_t c = 0; c < j; ++c) {
        P.job(L.off(K, j, c), b, nullptr, 0, b, b, 1.0, 0.0, JOB_C_F32);
        seg(pa, pb + c * bb);
      }
      P.gemm_end();
    }
    if (j == T - 1) break;
    std::vector<const float*> x(j + 1), col(T - j - 1);
    for (int64_t c = 0; c < j; ++c) x[c] = (const float*)L.off(K, j, c);
    x[j] = Wj;
    for (int64_t i = j + 1; i < T; ++i) col[i - j - 1] = (const float*)L.off(K, i, j);
    split(x, true, pb);
    split(col, false, pa);
    P.gemm_begin(1, kind, (double)(T - j - 1) * ((double)j * gemm + trmm));
    for (int64_t i = j + 1; i < T; ++i) {
      const uint16_t* Ai = pa + (i - j - 1) * bb;
      for (int64_t c = 0; c < j; ++c) {
        void* C = L.off(K, i, c);
        P.job(C, b, C, b, b, b, -1.0, 1.0, JOB_C_F32);
        seg(Ai, pb + c * bb);
      }
      P.job(L.off(K, i, j), b, nullptr, 0, b, b, -1.0, 0.0, JOB_C_F32);
      seg(Ai, pb + j * bb);
    }
    P.gemm_end();
  }
}

// describe_lauum_trace from split-bfloat16 planes: step k splits block row k of X = L^{-1}
// transposed (X_ki^T, i < k, and W_kk^T), which is both operand sets of its products
// X_ki^T X_kj, j <= i <= k.
void describe_lauum_trace_split(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  const int64_t b = L.b, T = L.T, bb = b * b, ps = w.pstride;
  const int np = prec == GPR_BF16X6 ? 3 : 2;
  const int kind = prec == GPR_BF16X6 ? GEMM_KIND_BF16X6_TRACE_T256 : GEMM_KIND_BF16X3_TRACE_T256;
  const double bd = (double)b;
  const double full = 2.0 * bd * bd * bd, half = bd * bd * (bd + 1.0), tri3 = bd * (bd + 1.0) * (bd + 2.0) / 3.0;
  uint16_t* const pb = w.pb;
  for (int64_t k = 0; k < T; ++k) {
    std::vector<const float*> x(k + 1);
    for (int64_t i = 0; i < k; ++i) x[i] = (const float*)L.off(K, k, i);
    x[k] = w.w32 + k * bb;
    P.kernel([=](hipStream_t s) {
      return launch_split_bf16_tiles(x.data(), (int64_t)x.size(), b, b, b, true, pb, ps, np, s);
    });
    const double kd = (double)k;
    P.gemm_begin(1, kind, kd * (kd - 1.0) / 2.0 * full + 2.0 * kd * half + tri3);
    for (int64_t i = 0; i <= k; ++i)
      for (int64_t j = 0; j <= i; ++j) {
        const int flags = (i == k ? JOB_TRACE_ALPHA : 0) | (i == j ? JOB_LOWER_ONLY : 0);
        P.job(nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, flags, (int)i, (int)j);
        P.seg(pb + i * bb, b, MODE_KC, pb + j * bb, b, MODE_KC, b, 0);
        P.segs.back().pstrideA = P.segs.back().pstrideB = ps;
      }
    P.gemm_end();
  }
}

// The split modes run the gradient's products from bfloat16 planes when the tiles suit the
// 256 x 256 kernels (with the products of the update), float32 otherwise.
bool grad_split(const TileLayout& L, int prec) { return is_bf16(prec) && bf16_tiled(L); }
void describe_grad_inverse(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  if (grad_split(L, prec)) describe_trtri_split(P, L, K, prec, w);
  else describe_trtri(P, L, K, prec, w);
}
void describe_grad_trace(Program& P, const TileLayout& L, void* K, int prec, const GradWs& w) {
  if (grad_split(L, prec)) describe_lauum_trace_split(P, L, K, prec, w);
  else describe_lauum_trace(P, L, K, prec, w);
}

GradWs carve_grad(Carve& c, const TileLayout& L, int prec) {
  GradWs w{};
  const int es = is_mixed(prec) ? 4 : 8;
  const size_t tiles = (size_t)(L.T > 1 ? L.T - 1 : 0) * L.b * L.b * es;
  const bool split = grad_split(L, prec);
  w.panel = split ? nullptr : c.take<char>(tiles);
  w.row = split ? nullptr : c.take<char>(tiles);
  w.w32 = is_mixed(prec) ? c.take<float>((size_t)L.T * L.b * L.b) : nullptr;
  if (split) {
    const int np = prec == GPR_BF16X6 ? 3 : 2;
    w.pstride = L.T * L.b * L.b;
    w.pa = c.take<uint16_t>((size_t)np * w.pstride);
    w.pb = c.take<uint16_t>((size_t)np * w.pstride);
  }
  w.partial_wg = trace_workgroups(L);
  w.partial = c.take<double>((size_t)w.partial_wg * 3 + 3);
  w.u = c.take<double>((size_t)(L.T * (L.T + 1) / 2) * L.b * L.b);
  w.apad = L.npad() > L.n ? c.take<double>(L.npad()) : nullptr;
  w.arena = c.take<char>(0);
  return w;
}

int grad_impl(const double* Z, int64_t d, HyperArg h, void* K, const TileLayout& L, int prec, const double* alpha,
              const int tr[3], double* grad, void* ws, size_t ws_bytes, hipStream_t st) {
  Carve c(ws);
  GradWs w = carve_grad(c, L, prec);
  const size_t fixed = c.off;
  const size_t cap = ws_bytes > fixed ? ws_bytes - fixed : 0;
  const bool mixed = is_mixed(prec);
  if (mixed) HIPCHK(launch_convert_f64_f32(L.winv(K, 0), w.w32, L.T * L.b * L.b, st));
  int rc = run_program([&](Program& P) { describe_grad_inverse(P, L, K, prec, w); }, w.arena, cap, st);
  if (rc) return rc;
  HIPCHK(launch_halfdist_tiles(Z, L.n, d, h, L.b, L.T, w.u, st));
  if (w.apad) {
    HIPCHK(launch_copy(w.apad, alpha, L.n * sizeof(double), st));
    HIPCHK(launch_fill_u64((unsigned long long*)(w.apad + L.n), 0ull, L.npad() - L.n, st));
    alpha = w.apad;
  }
  const TraceArgs ta{w.u, alpha, h, L.b, w.partial};
  int64_t nwg = 0;
  rc = run_program(
      [&](Program& P) {
        P.trace = &ta;
        P.trace_cap = w.partial_wg;
        describe_grad_trace(P, L, K, prec, w);
      },
      w.arena, cap, st, &nwg);
  if (rc) return rc;
  HIPCHK(launch_grad_finish(w.partial, nwg, h, L.npad() - L.n, tr[0], tr[1], tr[2], grad, st));
  return GPR_OK;
}

size_t grad_ws_bytes(const TileLayout& L, int prec) {
  Carve c(kSymWs);
  GradWs w = carve_grad(c, L, prec);
  Program P1, P2;
  describe_grad_inverse(P1, L, kSymK, prec, w);
  describe_grad_trace(P2, L, kSymK, prec, w);
  return c.off + std::max(arena_bytes_of(P1), arena_bytes_of(P2));
}

size_t var_ws_bytes(const TileLayout& L, int64_t m, int prec, bool full) {
  Carve c(kSymWs);
  VarWs w = carve_var(c, L, m, prec);
  Program P;
  describe_variance(P, L, kSymK, m, prec, w);
  if (full) describe_fullcov(P, L, m, prec, w, (double*)kSymOut);
  return c.off + arena_bytes_of(P);
}

size_t solve_ws_bytes(const TileLayout& L) {
  Carve c(nullptr);
  carve_solve(c, L);
  return c.off;
}

size_t predict_ws_bytes(int64_t n, int64_t m) {
  return (size_t)ceil_div(std::max<int64_t>(n, 1), kColsPerChunk) * std::max<int64_t>(m, 1) * 8 + 256;
}

size_t optimize_state_bytes(int64_t n, int steps) {
  Carve c(nullptr);
  c.take<double>(3);            // theta
  c.take<double>(7);            // adam state
  c.take<double>(3);            // grad
  c.take<double>(steps + 1);    // nlml trace
  c.take<double>(n);            // alpha
  return c.off + 256;
}

// The executor's scheduling code on the host (gpr_dag_check): the atomics are the
// compiler's, the clock counts nanoseconds, a wait yields the thread.
struct DagHostOps {
  static int fetch_add_relaxed(int32_t* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
  static int fetch_add_acq_rel(int32_t* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
  static int fetch_add_release(int32_t* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELEASE); }
  static int load_acquire(int32_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
  static int load_relaxed(int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
  static void fence_acquire() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
  static void store_release(int32_t* p, int v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
  static void cas_relaxed(int32_t* p, int expected, int desired) {
    __atomic_compare_exchange_n(p, &expected, desired, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
  }
  static uint64_t clock() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
  }
  static void pause() { std::this_thread::yield(); }
};
typedef DagCore<DagHostOps> HostCore;

// Largest job-table upload of any call on a problem of this size (staging slot size).
size_t table_bytes(const TileLayout& L, int64_t m, int prec) {
  size_t t = chol_sizes(L, prec).arena;
  {
    Carve c(kSymWs);
    VarWs w = carve_var(c, L, m, prec);
    Program P;
    describe_variance(P, L, kSymK, m, prec, w);
    describe_fullcov(P, L, m, prec, w, (double*)kSymOut);
    t = std::max(t, arena_bytes_of(P));
  }
  {
    Carve c(kSymWs);
    GradWs w = carve_grad(c, L, prec);
    Program P1, P2;
    describe_grad_inverse(P1, L, kSymK, prec, w);
    describe_grad_trace(P2, L, kSymK, prec, w);
    t = std::max(t, std::max(arena_bytes_of(P1), arena_bytes_of(P2)));
  }
  return t;
}

size_t chol_ws_bytes(const TileLayout& L, int prec) {
  CholSizes s = chol_sizes(L, prec);
  return s.fixed + 256 + s.arena;
}

// The task-graph executor gives up when no task has finished for this long.
constexpr double kDagWaitLimitSeconds = 10.0;

// The factorisation as a task graph on the device; *ran = false when this problem has no
// task form (the caller then uses the streams).
int chol_graph(void* K, const TileLayout& L, int prec, const CholWs& w, hipStream_t st, bool* ran) {
  *ran = false;
  Program P;
  DagRecord R;
  P.dagr = &R;
  describe_cholesky_graph(P, L, K, prec, w);
  if (!R.ok || R.tasks.empty() || (int64_t)R.tasks.size() > w.dag_ntasks) return GPR_OK;
  std::vector<int32_t> succ;
  if (!dag_edges(R, succ, dag_max_succ(R.tasks.size()))) return GPR_OK;
  DevRes* D = nullptr;
  int rc = current_res(&D);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(D->mu);
    if (D->dag_slots <= 0) HIPCHK(dag_slots(&D->dag_slots));
  }
  std::vector<void*> dev;
  rc = upload_parts({{P.jobs.data(), P.jobs.size() * sizeof(GemmJob)}, {P.segs.data(), P.segs.size() * sizeof(GemmSeg)},
                     {R.tasks.data(), R.tasks.size() * sizeof(DagTask)}, {succ.data(), succ.size() * sizeof(int32_t)},
                     {R.ops.data(), R.ops.size() * sizeof(DagOp)}},
                    w.arena, w.arena_cap, st, dev);
  if (rc) return rc;
  const int nt = (int)R.tasks.size();
  unsigned long long* info = w.info;
  HIPCHK(launch_fill_u64(info, ~0ull, 2, st));
  HIPCHK(launch_dag((const DagTask*)dev[2], nt, (const int32_t*)dev[3], (const DagOp*)dev[4], (const GemmJob*)dev[0],
                    (const GemmSeg*)dev[1], w.dag_state, info, kDagWaitLimitSeconds, D->dag_slots, st));
  HIPCHK(launch_copy(info + 2, info, 2 * sizeof(unsigned long long), st));
  *ran = true;
  return GPR_OK;
}

int chol_impl(void* K, const TileLayout& L, int prec, void* ws, size_t ws_bytes, unsigned long long** info_out,
              hipStream_t st) {
  CholWs w = carve_chol(ws, L, prec, ws_bytes);
  if (info_out) *info_out = w.info + 2;   // set by the factorisation's last kernel

  const int mode = g_schedule.load(std::memory_order_relaxed);
  if (mode == GPR_SCHEDULE_DEVICE && prec == GPR_FP64) {
    bool ran = false;
    int rc = chol_graph(K, L, prec, w, st, &ran);
    if (rc || ran) return rc;
  }
  const bool la = mode != GPR_SCHEDULE_STREAM;
  if (!la)
    return run_program([&](Program& P) { describe_cholesky(P, L, K, prec, w, false); }, w.arena, w.arena_cap, st);
  // the auxiliary stream and events are shared by all calls on this device: serialise
  // factorisations so that one call's events are not re-recorded by another
  DevRes* R = nullptr;
  int rc = current_res(&R);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(R->chol_mu);
  return run_program([&](Program& P) { describe_cholesky(P, L, K, prec, w, true); }, w.arena, w.arena_cap, st,
                     nullptr, chol_events_needed(L.T));
}

}  // namespace

// ================================================================ C-ABI
extern "C" {

GPR_API int gpr_version(void) { return (1 << 16) | (0 << 8) | 0; }

GPR_API const char* gpr_last_error(void) { return g_err; }

GPR_API int gpr_init(int64_t n, int64_t m, int64_t tile, int prec) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if (n < 0 || m < 0) return fail(GPR_ERR_SHAPE, "need n, m >= 0");
  if (n > 0 && (rc = check_shape(n, tile))) return rc;
  size_t tb = kMinSlotBytes;
  int nev = chol_events_needed(1);
  if (n > 0) {
    const TileLayout L = layout_of(n, tile, prec);
    tb = std::max(tb, table_bytes(L, m, prec));
    nev = chol_events_needed(L.T);
  }
  DevRes* R = nullptr;
  if ((rc = current_res(&R))) return rc;
  HIPCHK(scratch_setup(nullptr));   // address of this device's scratch for gpr_predict_noalloc
  std::lock_guard<std::mutex> lk(R->mu);
  if ((rc = ensure_aux(R, nev))) return rc;
  return grow_slots(R, tb);
}

GPR_API int gpr_set_lookahead(int on) {
  g_schedule.store(on != 0 ? GPR_SCHEDULE_LOOKAHEAD : GPR_SCHEDULE_STREAM, std::memory_order_relaxed);
  return GPR_OK;
}

GPR_API int gpr_set_schedule(int mode) {
  if (mode < GPR_SCHEDULE_STREAM || mode > GPR_SCHEDULE_DEVICE) return fail(GPR_ERR_ARG, "unknown schedule %d", mode);
  g_schedule.store(mode, std::memory_order_relaxed);
  return GPR_OK;
}

GPR_API int gpr_tiles_bytes(int64_t n, int64_t tile, int prec, size_t* bytes) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (!bytes) return fail(GPR_ERR_ARG, "bytes is NULL");
  *bytes = layout_of(n, tile, prec).total_bytes();
  return GPR_OK;
}

GPR_API int gpr_workspace_size(int64_t n, int64_t m, int64_t d, int64_t tile, int prec, size_t* bytes) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (m < 0 || d < 1) return fail(GPR_ERR_SHAPE, "need m >= 0 and d >= 1");
  if (!bytes) return fail(GPR_ERR_ARG, "bytes is NULL");
  const TileLayout L = layout_of(n, tile, prec);
  size_t need = chol_ws_bytes(L, prec);
  need = std::max(need, solve_ws_bytes(L));
  need = std::max(need, predict_ws_bytes(n, m));
  need = std::max(need, var_ws_bytes(L, m, prec, true));
  need = std::max(need, grad_ws_bytes(L, prec));
  // gpr_optimize keeps its state in front of the per-step workspaces
  const size_t step = std::max(std::max(chol_ws_bytes(L, prec), solve_ws_bytes(L)), grad_ws_bytes(L, prec));
  need = std::max(need, optimize_state_bytes(n, 4096) + step);
  *bytes = need + 4096;
  return GPR_OK;
}

GPR_API int gpr_assemble(const double* Z, int64_t n, int64_t d, gpr_hyper_t h, int64_t tile, int prec, void* K_tiles,
                         void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if ((rc = check_hyper(h))) return rc;
  if (d < 1) return fail(GPR_ERR_SHAPE, "d must be >= 1");
  if (n == 0) return GPR_OK;
  if (!Z || !K_tiles) return fail(GPR_ERR_ARG, "null pointer");
  HIPCHK(launch_assemble_tiles(Z, d, harg(h), layout_of(n, tile, prec), K_tiles, (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_cholesky(void* K_tiles, int64_t n, int64_t tile, int prec, void* ws, size_t ws_bytes, int64_t* info,
                         void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (n == 0) {
    if (info) *info = 0;
    return GPR_OK;
  }
  if (!K_tiles || !ws) return fail(GPR_ERR_ARG, "null pointer");
  const TileLayout L = layout_of(n, tile, prec);
  if (ws_bytes < chol_ws_bytes(L, prec))
    return fail(GPR_ERR_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, chol_ws_bytes(L, prec));
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* dinfo = nullptr;
  if ((rc = chol_impl(K_tiles, L, prec, ws, ws_bytes, &dinfo, st))) return rc;
  if (info) {
    unsigned long long hinfo[1] = {0};
    HIPCHK(hipMemcpyAsync(hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hinfo[0] == DAG_ABORT_INFO) {
      *info = 0;
      return fail(GPR_ERR_HIP, "device task graph gave up: a task waited longer than %.0f s", kDagWaitLimitSeconds);
    }
    if (hinfo[0] != std::numeric_limits<unsigned long long>::max()) {
      *info = (int64_t)hinfo[0];
      return fail(GPR_ERR_NOT_SPD, "matrix is not positive definite: pivot %lld", (long long)hinfo[0]);
    }
    *info = 0;
  }
  return GPR_OK;
}

GPR_API int gpr_solve(const void* L_tiles, const double* Z, int64_t n, int64_t d, gpr_hyper_t h, int64_t tile, int prec,
                      const double* y, double* alpha, int refine_sweeps, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (refine_sweeps < 0) refine_sweeps = default_sweeps(prec);
  if (n == 0) return GPR_OK;
  if (!L_tiles || !y || !alpha || !ws) return fail(GPR_ERR_ARG, "null pointer");
  if (y == alpha) return fail(GPR_ERR_ARG, "alpha may not alias y");
  if (refine_sweeps > 0) {
    if ((rc = check_hyper(h))) return rc;
    if (!Z || d < 1) return fail(GPR_ERR_ARG, "refinement needs Z and d >= 1");
  }
  const TileLayout L = layout_of(n, tile, prec);
  if (ws_bytes < solve_ws_bytes(L)) return fail(GPR_ERR_WORKSPACE, "workspace too small");
  Carve c(ws);
  SolveWs w = carve_solve(c, L);
  return solve_impl(L, L_tiles, Z, d, harg(h), y, alpha, refine_sweeps, w, (hipStream_t)stream);
}

GPR_API int gpr_predict(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                        const double* alpha, double* mean, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_hyper(h))) return rc;
  if (n < 0 || m < 0 || d < 1) return fail(GPR_ERR_SHAPE, "need n, m >= 0 and d >= 1");
  if (m == 0) return GPR_OK;
  if (!Zs || !mean) return fail(GPR_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    HIPCHK(hipMemsetAsync(mean, 0, m * sizeof(double), st));
    return GPR_OK;
  }
  if (!Z || !alpha || !ws) return fail(GPR_ERR_ARG, "null pointer");
  if (ws_bytes < predict_ws_bytes(n, m)) return fail(GPR_ERR_WORKSPACE, "workspace too small");
  double* partial = (double*)ws;
  HIPCHK(launch_kmatvec_partial(Zs, m, Z, n, d, harg(h), alpha, partial, kColsPerChunk, st));
  HIPCHK(launch_reduce_partials(partial, ceil_div(n, kColsPerChunk), m, 1.0, nullptr, 0.0, mean, st));
  return GPR_OK;
}

GPR_API int gpr_predict_noalloc(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                                const double* alpha, double* mean, void* stream) {
  int rc;
  if ((rc = check_hyper(h))) return rc;
  if (n < 0 || m < 0 || d < 1) return fail(GPR_ERR_SHAPE, "need n, m >= 0 and d >= 1");
  if (m == 0) return GPR_OK;
  if (!Zs || !mean) return fail(GPR_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    HIPCHK(launch_fill_u64((unsigned long long*)mean, 0ull, m, st));   // +0.0 bits
    return GPR_OK;
  }
  if (!Z || !alpha) return fail(GPR_ERR_ARG, "null pointer");
  const int64_t nch = ceil_div(n, kColsPerChunk);
  if (m > kScratchDoubles / nch)
    return fail(GPR_ERR_WORKSPACE,
                "gpr_predict_noalloc: ceil(n / %lld) * m = %lld partial sums exceed the fixed scratch of %lld",
                (long long)kColsPerChunk, (long long)(nch * m), (long long)kScratchDoubles);
  double* partial = nullptr;
  HIPCHK(scratch_setup(&partial));
  HIPCHK(launch_kmatvec_partial(Zs, m, Z, n, d, harg(h), alpha, partial, kColsPerChunk, st));
  HIPCHK(launch_reduce_partials(partial, nch, m, 1.0, nullptr, 0.0, mean, st));
  return GPR_OK;
}

GPR_API int gpr_predict_var(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                            const void* L_tiles, int64_t tile, int prec, int full_cov, int add_noise, double* out,
                            void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if ((rc = check_hyper(h))) return rc;
  if (m < 0 || d < 1) return fail(GPR_ERR_SHAPE, "need m >= 0 and d >= 1");
  if (m == 0) return GPR_OK;
  if (!Zs || !out) return fail(GPR_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const HyperArg ha = harg(h);
  if (n == 0) {
    // no data: the posterior is the prior
    if (full_cov) HIPCHK(launch_assemble_dense(Zs, m, Zs, m, d, ha, add_noise, out, m, 0, st));
    else {
      Carve c(ws);
      (void)c;
      HIPCHK(launch_var_finish(nullptr, 0, m, ha, add_noise, out, st));
    }
    return GPR_OK;
  }
  if (!Z || !L_tiles || !ws) return fail(GPR_ERR_ARG, "null pointer");
  const TileLayout L = layout_of(n, tile, prec);
  const size_t need = var_ws_bytes(L, m, prec, full_cov != 0);
  if (ws_bytes < need) return fail(GPR_ERR_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, need);
  Carve c(ws);
  VarWs w = carve_var(c, L, m, prec);
  const bool mixed = is_mixed(prec);
  void* K = const_cast<void*>(L_tiles);
  if (mixed) HIPCHK(launch_convert_f64_f32(L.winv(K, 0), w.w32, L.T * L.b * L.b, st));
  HIPCHK(launch_assemble_dense(Z, n, Zs, m, d, ha, 0, w.V, m, mixed ? 1 : 0, st));
  if (L.npad() > n) {
    // the padding's rows of the cross-covariance are zero
    const size_t es = mixed ? 4 : 8;
    HIPCHK(launch_zero((char*)w.V + (size_t)n * m * es, (size_t)(L.npad() - n) * m * es, st));
  }
  if (full_cov) HIPCHK(launch_assemble_dense(Zs, m, Zs, m, d, ha, add_noise, out, m, 0, st));
  rc = run_program(
      [&](Program& P) {
        describe_variance(P, L, L_tiles, m, prec, w);
        if (full_cov) describe_fullcov(P, L, m, prec, w, out);
      },
      w.arena, ws_bytes - c.off, st);
  if (rc) return rc;
  if (!full_cov) {
    HIPCHK(launch_colsq_partial(w.V, mixed ? 1 : 0, m, n, m, w.partial, kRowsPerChunk, st));
    HIPCHK(launch_var_finish(w.partial, ceil_div(n, kRowsPerChunk), m, ha, add_noise, out, st));
  }
  return GPR_OK;
}

GPR_API int gpr_nlml(const void* L_tiles, int64_t n, int64_t tile, int prec, const double* y, const double* alpha,
                     double* nlml, void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (!nlml) return fail(GPR_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    HIPCHK(hipMemsetAsync(nlml, 0, sizeof(double), st));
    return GPR_OK;
  }
  if (!L_tiles || !y || !alpha) return fail(GPR_ERR_ARG, "null pointer");
  const TileLayout L = layout_of(n, tile, prec);
  HIPCHK(launch_nlml(L.diag(const_cast<void*>(L_tiles), 0), L.b, L.n, y, alpha, nlml, st));
  return GPR_OK;
}

GPR_API int gpr_nlml_grad(const double* Z, int64_t n, int64_t d, gpr_hyper_t h, void* L_tiles, int64_t tile, int prec,
                          const double* alpha, const int* trainable, double* grad_log, void* ws, size_t ws_bytes,
                          void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if ((rc = check_hyper(h))) return rc;
  if (d < 1) return fail(GPR_ERR_SHAPE, "d must be >= 1");
  if (!grad_log) return fail(GPR_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    HIPCHK(hipMemsetAsync(grad_log, 0, 3 * sizeof(double), st));
    return GPR_OK;
  }
  if (!Z || !L_tiles || !alpha || !ws) return fail(GPR_ERR_ARG, "null pointer");
  const TileLayout L = layout_of(n, tile, prec);
  if (ws_bytes < grad_ws_bytes(L, prec)) return fail(GPR_ERR_WORKSPACE, "workspace too small");
  int tr[3] = {1, 1, 1};
  if (trainable)
    for (int k = 0; k < 3; ++k) tr[k] = trainable[k] != 0;
  return grad_impl(Z, d, harg(h), L_tiles, L, prec, alpha, tr, grad_log, ws, ws_bytes, st);
}

GPR_API int gpr_optimize(const double* Z, const double* y, int64_t n, int64_t d, int64_t tile, int prec, int kernel,
                         double* theta_log, const int* trainable, int steps, double lr, double beta1, double beta2,
                         double eps, double* adam_state, double* nlml_trace, void* K_tiles, void* ws,
                         size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if (kernel < GPR_KERNEL_SE || kernel > GPR_KERNEL_MATERN52) return fail(GPR_ERR_ARG, "unknown kernel %d", kernel);
  if ((rc = check_shape(n, tile))) return rc;
  if (d < 1 || n < 1) return fail(GPR_ERR_SHAPE, "need n >= 1 and d >= 1");
  if (steps < 0 || steps > 4095) return fail(GPR_ERR_ARG, "steps must be in [0, 4095]");
  if (!Z || !y || !theta_log || !adam_state || !K_tiles || !ws) return fail(GPR_ERR_ARG, "null pointer");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(theta_log[k])) return fail(GPR_ERR_ARG, "theta_log must be finite");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
    return fail(GPR_ERR_ARG, "bad Adam parameters");
  const TileLayout L = layout_of(n, tile, prec);
  const size_t state = optimize_state_bytes(n, 4096);
  const size_t step_need = std::max(std::max(chol_ws_bytes(L, prec), solve_ws_bytes(L)), grad_ws_bytes(L, prec));
  if (ws_bytes < state + step_need) return fail(GPR_ERR_WORKSPACE, "workspace too small");
  int tr[3] = {1, 1, 1};
  if (trainable)
    for (int k = 0; k < 3; ++k) tr[k] = trainable[k] != 0;
  hipStream_t st = (hipStream_t)stream;
  Carve c(ws);
  double* dtheta = c.take<double>(3);
  double* dstate = c.take<double>(7);
  double* dgrad = c.take<double>(3);
  double* dtrace = c.take<double>(4097);
  double* dalpha = c.take<double>(n);
  void* ws2 = (char*)ws + state;
  const size_t ws2_bytes = ws_bytes - state;
  HIPCHK(hipMemcpyAsync(dtheta, theta_log, 3 * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dstate, adam_state, 7 * sizeof(double), hipMemcpyHostToDevice, st));
  const HyperArg hd{0.0, 0.0, 0.0, dtheta, kernel};
  unsigned long long* dinfo = nullptr;
  Carve cs(ws2);
  for (int s = 0; s <= steps; ++s) {
    HIPCHK(launch_assemble_tiles(Z, d, hd, L, K_tiles, st));
    if ((rc = chol_impl(K_tiles, L, prec, ws2, ws2_bytes, &dinfo, st))) return rc;
    {
      Carve c2(ws2);
      c2.take<unsigned long long>(32);   // keep the factorisation's info word intact
      SolveWs sw = carve_solve(c2, L);
      if ((rc = solve_impl(L, K_tiles, Z, d, hd, y, dalpha, default_sweeps(prec), sw, st))) return rc;
    }
    HIPCHK(launch_nlml(L.diag(K_tiles, 0), L.b, L.n, y, dalpha, dtrace + s, st));
    if (s == steps) break;
    {
      Carve c2(ws2);
      c2.take<unsigned long long>(32);
      void* gws = c2.take<char>(0);
      if ((rc = grad_impl(Z, d, hd, K_tiles, L, prec, dalpha, tr, dgrad, gws, ws2_bytes - c2.off, st))) return rc;
    }
    HIPCHK(launch_adam3(dtheta, dstate, dgrad, lr, beta1, beta2, eps, tr[0], tr[1], tr[2], st));
  }
  unsigned long long hinfo = 0;
  HIPCHK(hipMemcpyAsync(theta_log, dtheta, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(adam_state, dstate, 7 * sizeof(double), hipMemcpyDeviceToHost, st));
  if (nlml_trace) HIPCHK(hipMemcpyAsync(nlml_trace, dtrace, (steps + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hinfo != std::numeric_limits<unsigned long long>::max())
    return fail(GPR_ERR_NOT_SPD, "covariance lost positive definiteness during optimisation (pivot %lld)",
                (long long)hinfo);
  return GPR_OK;
}

GPR_API int gpr_split_bf16x3(const float* x, int64_t count, void* hi, void* mid, void* lo, void* stream) {
  if (count < 0) return fail(GPR_ERR_SHAPE, "negative count");
  if (count == 0) return GPR_OK;
  if (!x || !hi || !mid || !lo) return fail(GPR_ERR_ARG, "null pointer");
  HIPCHK(launch_split_bf16x3(x, count, hi, mid, lo, (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_stats_workspace(int64_t nsub, size_t* bytes) {
  if (nsub < 2 || nsub > 4096 || !bytes) return fail(GPR_ERR_ARG, "need 2 <= nsub <= 4096 and bytes");
  *bytes = (size_t)stats_sort_len(nsub) * sizeof(double) + 256;
  return GPR_OK;
}

GPR_API int gpr_summary_stats(const double* Z_raw, const double* Z_std, const double* y_raw, int64_t n, int64_t d,
                              const int64_t* sub_idx, int64_t nsub, double* stats64, float* stats32, void* ws,
                              size_t ws_bytes, void* stream) {
  if (n < 1 || d < 1 || d > 256) return fail(GPR_ERR_SHAPE, "need n >= 1 and 1 <= d <= 256");
  if (nsub < 2 || nsub > 4096 || nsub > n) return fail(GPR_ERR_SHAPE, "need 2 <= nsub <= min(n, 4096)");
  if (!Z_raw || !Z_std || !y_raw || !sub_idx || !ws || (!stats64 && !stats32)) return fail(GPR_ERR_ARG, "null pointer");
  if (ws_bytes < (size_t)stats_sort_len(nsub) * sizeof(double)) return fail(GPR_ERR_WORKSPACE, "workspace too small");
  HIPCHK(launch_summary_stats(Z_raw, Z_std, y_raw, n, d, sub_idx, nsub, (double*)ws, stats64, stats32,
                              (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_mlp_nparams(void) { return mlp_nparams(); }

GPR_API int gpr_mlp_workspace(int64_t batch, size_t* bytes) {
  if (batch < 1 || batch > 65536 || !bytes) return fail(GPR_ERR_ARG, "need 1 <= batch <= 65536 and bytes");
  *bytes = (mlp_act_floats((int)batch) + (size_t)mlp_nparams()) * sizeof(float) + 512;
  return GPR_OK;
}

static int mlp_check(int64_t batch, void* ws, size_t ws_bytes) {
  if (batch < 1 || batch > 65536) return fail(GPR_ERR_SHAPE, "need 1 <= batch <= 65536");
  if (!ws) return fail(GPR_ERR_ARG, "null workspace");
  if (ws_bytes < (mlp_act_floats((int)batch) + (size_t)mlp_nparams()) * sizeof(float))
    return fail(GPR_ERR_WORKSPACE, "workspace too small");
  return GPR_OK;
}

GPR_API int gpr_mlp_forward(const float* params, const float* X, int64_t batch, float* out, void* ws, size_t ws_bytes,
                            void* stream) {
  int rc;
  if ((rc = mlp_check(batch, ws, ws_bytes))) return rc;
  if (!params || !X || !out) return fail(GPR_ERR_ARG, "null pointer");
  HIPCHK(launch_mlp(const_cast<float*>(params), nullptr, nullptr, nullptr, X, nullptr, out, nullptr, (float*)ws,
                    (int)batch, 0, 0.f, 0.f, 0.f, 0.f, 0, (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_mlp_loss_grad(const float* params, const float* X, const float* Y, int64_t batch, float* loss,
                              float* grad, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = mlp_check(batch, ws, ws_bytes))) return rc;
  if (!params || !X || !Y || !grad) return fail(GPR_ERR_ARG, "null pointer");
  HIPCHK(launch_mlp(const_cast<float*>(params), nullptr, nullptr, grad, X, Y, nullptr, loss, (float*)ws, (int)batch, 1,
                    0.f, 0.f, 0.f, 0.f, 0, (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_mlp_train_step(float* params, float* adam_m, float* adam_v, int t, const float* X, const float* Y,
                               int64_t batch, float lr, float beta1, float beta2, float eps, float* loss, void* ws,
                               size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = mlp_check(batch, ws, ws_bytes))) return rc;
  if (!params || !adam_m || !adam_v || !X || !Y) return fail(GPR_ERR_ARG, "null pointer");
  if (t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
    return fail(GPR_ERR_ARG, "bad Adam parameters");
  float* grad = (float*)ws + mlp_act_floats((int)batch);
  HIPCHK(launch_mlp(params, adam_m, adam_v, grad, X, Y, nullptr, loss, (float*)ws, (int)batch, 2, lr, beta1, beta2,
                    eps, t, (hipStream_t)stream));
  return GPR_OK;
}

GPR_API int gpr_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  g_timing.on = on != 0;
  return GPR_OK;
}

GPR_API int gpr_timing_read(int kind, int64_t* launches, double* total_ms, double* algo_flops) {
  if (!launches || !total_ms || !algo_flops) return fail(GPR_ERR_ARG, "null pointer");
  if (kind < 0 || kind > 11) return fail(GPR_ERR_ARG, "kind must be 0..11");
  std::lock_guard<std::mutex> lk(g_timing.mu);
  int64_t cnt = 0;
  double ms = 0.0, fl = 0.0;
  std::vector<TimingLog::Rec> keep;
  for (auto& r : g_timing.recs) {
    if (r.kind != kind) {
      keep.push_back(r);
      continue;
    }
    HIPCHK(hipEventSynchronize(r.b));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    fl += r.flops;
    ++cnt;
    g_timing.pool.push_back(r.a);
    g_timing.pool.push_back(r.b);
  }
  g_timing.recs.swap(keep);
  *launches = cnt;
  *total_ms = ms;
  *algo_flops = fl;
  return GPR_OK;
}

GPR_API int gpr_cholesky_schedule_check(int64_t n, int64_t tile, int prec, int64_t omit_event, int64_t* report) {
  int rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (!report) return fail(GPR_ERR_ARG, "report is NULL");
  if (n == 0) {
    for (int i = 0; i < 8; ++i) report[i] = 0;
    return GPR_OK;
  }
  // symbolic addresses: the trace pass only compares them, nothing is dereferenced
  const TileLayout L = layout_of(n, tile, prec);
  void* K = kSymK;
  const size_t wsb = chol_ws_bytes(L, prec);
  const CholWs w = carve_chol(kSymWs, L, prec, wsb);
  AccessLog log;
  Program P;
  P.alog = &log;
  describe_cholesky(P, L, K, prec, w, true);
  ScheduleReport r;
  check_schedule(log, (int)omit_event, r);
  report[0] = r.launches;
  report[1] = r.on_stream[0];
  report[2] = r.on_stream[1];
  report[3] = r.waits;
  report[4] = r.concurrent_pairs;
  report[5] = r.conflicts;
  report[6] = r.unannotated;
  report[7] = r.early_waits;
  return GPR_OK;
}

GPR_API int gpr_dag_check(int64_t n, int64_t tile, int threads, int64_t withhold, double limit_ms, int64_t* report) {
  int rc;
  if ((rc = check_shape(n, tile))) return rc;
  if (!report || threads < 1 || threads > 4096 || !(limit_ms > 0)) return fail(GPR_ERR_ARG, "bad arguments");
  for (int i = 0; i < 9; ++i) report[i] = 0;
  if (n == 0) return GPR_OK;
  const TileLayout L = layout_of(n, tile, GPR_FP64);
  void* K = kSymK;
  const size_t wsb = chol_ws_bytes(L, GPR_FP64);
  const CholWs w = carve_chol(kSymWs, L, GPR_FP64, wsb);
  Program P;
  DagRecord R;
  P.dagr = &R;
  describe_cholesky_graph(P, L, K, GPR_FP64, w);
  if (!R.ok) return fail(GPR_ERR_ARG, "this problem has no task-graph form");
  std::vector<int32_t> succ;
  if (!dag_edges(R, succ, dag_max_succ(R.tasks.size()))) return fail(GPR_ERR_ARG, "too many edges");
  const int nt = (int)R.tasks.size();
  if (withhold >= nt) return fail(GPR_ERR_ARG, "withhold >= number of tasks");
  if (withhold <= -2) {
    // drop edge number -2 - withhold (successor-list order) before the checks
    const int64_t e = -2 - withhold;
    if (e >= (int64_t)succ.size()) return fail(GPR_ERR_ARG, "no such edge");
    int u = 0;
    while (!(R.tasks[u].succ0 <= e && e < R.tasks[u].succ0 + R.tasks[u].nsucc)) ++u;
    const int t = succ[e];
    --R.tasks[t].npred;
    for (int64_t q = e; q + 1 < R.tasks[u].succ0 + R.tasks[u].nsucc; ++q) succ[q] = succ[q + 1];
    --R.tasks[u].nsucc;
  }
  std::vector<std::vector<int32_t>> preds(nt);
  for (int u = 0; u < nt; ++u)
    for (int q = 0; q < R.tasks[u].nsucc; ++q) preds[succ[R.tasks[u].succ0 + q]].push_back(u);
  // Independent of how the edges were derived: every pair of tasks whose exact byte ranges
  // overlap, one of them writing, must be ordered by a path of edges (graphs of up to 4096
  // tasks; -1 above that).  Edges only run from earlier to later tasks.
  int64_t unordered = -1;
  if (nt <= 4096) {
    unordered = 0;
    const int words = (nt + 63) / 64;
    std::vector<uint64_t> anc((size_t)nt * words, 0);
    for (int t = 0; t < nt; ++t)
      for (int32_t p : preds[t]) {
        if (p >= t) ++unordered;   // an edge against the issue order
        for (int q = 0; q < words; ++q) anc[(size_t)t * words + q] |= anc[(size_t)p * words + q];
        anc[(size_t)t * words + p / 64] |= 1ull << (p % 64);
      }
    auto overlap = [](const std::vector<Span>& a, const std::vector<Span>& b) {
      for (const Span& x : a)
        for (const Span& y : b)
          if (x.lo < y.hi && y.lo < x.hi) return true;
      return false;
    };
    for (int t = 0; t < nt; ++t)
      for (int u = 0; u < t; ++u) {
        if (anc[(size_t)t * words + u / 64] >> (u % 64) & 1) continue;
        if (overlap(R.wr[u], R.rd[t]) || overlap(R.wr[u], R.wr[t]) || overlap(R.rd[u], R.wr[t])) ++unordered;
      }
  }
  std::vector<int32_t> state(dag_state_ints(nt), 0);
  DagState S = dag_state_at(state.data(), nt);
  for (int t = 0; t < nt; ++t) {
    S.pending[t] = R.tasks[t].npred + (t == withhold ? 1 : 0);
    S.remaining[t] = R.tasks[t].nitems;
    S.rq0[t] = S.rq1[t] = -1;
  }
  std::vector<std::atomic<int64_t>> runs(R.items);   // how often each item ran (exactly once)
  for (int t = 0; t < nt; ++t)
    if (S.pending[t] == 0) HostCore::publish(R.tasks.data(), S, t);
  std::atomic<int64_t> ran{0}, violations{0}, returned{0};
  const uint64_t limit = (uint64_t)(limit_ms * 1.0e6);   // the host clock counts nanoseconds
  std::atomic<int> next_lane{0};
  auto worker = [&]() {
    const int lane = next_lane.fetch_add(1) % DAG_LANES;
    int last = -1;
    uint64_t since = 0;
    while (true) {
      int t = 0, idx = 0, q = 0, h = 0;
      if (!HostCore::try_claim(R.tasks.data(), S, lane, t, idx, q, h)) {
        if (!HostCore::keep_waiting(S, last, since, limit)) break;
        continue;
      }
      DagHostOps::fence_acquire();   // as the device executor before an item
      runs[R.tasks[t].item0 + idx].fetch_add(1);
      for (int32_t p : preds[t])
        if (DagHostOps::load_acquire(&S.remaining[p]) != 0) violations.fetch_add(1);
      ran.fetch_add(1);
      HostCore::finish(R.tasks.data(), succ.data(), S, t);
    }
    returned.fetch_add(1);
  };
  std::vector<std::thread> pool;
  for (int i = 0; i < threads; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  report[0] = nt;
  report[1] = R.items;
  report[2] = (int64_t)succ.size();
  report[3] = ran.load();
  for (auto& r : runs)
    if (r.load() != 1 && !S.ctl->abort) ++report[4];   // an item lost or run twice
  report[4] = violations.load();
  report[5] = S.ctl->abort;
  report[6] = S.ctl->timed_out;
  report[7] = returned.load();
  report[8] = unordered;
  return GPR_OK;
}

GPR_API int gpr_cholesky_census(int64_t T, int64_t* counts) {
  if (T < 0 || !counts) return fail(GPR_ERR_ARG, "bad arguments");
  // count the tile tasks exactly as describe_cholesky issues them (b = 1 keeps it cheap)
  int64_t potrf = 0, trsm = 0, syrk = 0, gemm = 0;
  for (int64_t k = 0; k < T; ++k) {
    ++potrf;
    if (k == T - 1) break;
    trsm += T - k - 1;
    for (int64_t nn = k + 1; nn < T; ++nn)
      for (int64_t m = nn; m < T; ++m) (m == nn ? syrk : gemm) += 1;
  }
  counts[0] = potrf;
  counts[1] = trsm;
  counts[2] = syrk;
  counts[3] = gemm;
  return GPR_OK;
}

}  // extern "C"
