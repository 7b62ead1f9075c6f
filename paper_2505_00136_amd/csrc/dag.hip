// Persistent executor of the factorisation's task graph on the device (see dag.h).
//
// One workgroup of 512 threads per slot, as many as fit on the device (two per CU with
// the tile-product kernels' 67.6 KB of LDS).  Thread 0 takes the next item of a ready task
// (or, when none is ready, polls until one is, giving up when no task has finished for
// longer than the time limit); the whole workgroup runs it -- a 128 x 128 macro tile of a
// tile product with the same code as the launch-per-step kernels, so the results are the
// same bits, or a piece of a copy, transpose, fill or diagonal-block factorisation.  Every
// thread makes its writes visible at device scope (a release fence) before thread 0
// counts the item as finished; the workgroup that finishes a task's last item releases its
// successors.  All counters and queue slots are accessed with device-scope atomics, so a
// poll is never served from a stale cache line of another XCD.
#include "common.h"
#include "dag.h"
#include "gemm_device.h"
#include "kernels.h"
#include "potrf_device.h"

namespace gpr {

struct DagDeviceOps {
  static __device__ int fetch_add_relaxed(int32_t* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ int fetch_add_acq_rel(int32_t* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ int fetch_add_release(int32_t* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ int load_relaxed(int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
  static __device__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
  static __device__ void store_release(int32_t* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ void cas_relaxed(int32_t* p, int expected, int desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ uint64_t clock() { return wall_clock64(); }   // constant-rate counter
  static __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
};
typedef DagCore<DagDeviceOps> DevCore;

constexpr int DAG_THREADS = 512;
constexpr int DAG_WN = 4;   // the tile-product wave layout of the launch-per-step kernels
static_assert(Shape<DAG_WN>::THREADS == DAG_THREADS, "workgroup shape");
constexpr int DAG_SMEM = Chunk<double>::SMEM;
static_assert(potrf_block_smem<64>() <= DAG_SMEM && 64 * 65 * 8 <= DAG_SMEM, "LDS of the task kinds");

struct DagArgs {
  const DagTask* tasks;
  const int32_t* succ;
  const DagOp* ops;
  const GemmJob* jobs;
  const GemmSeg* segs;
  int32_t* state;   // dag_state_at(state, ntasks)
  unsigned long long* info;
  int ntasks;
  uint64_t limit;   // wall-clock ticks without a finished task after which the run gives up
};

__global__ void dag_reset_kernel(DagArgs a) {
  DagState S = dag_state_at(a.state, a.ntasks);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.ntasks) {
    S.pending[i] = a.tasks[i].npred;
    S.remaining[i] = a.tasks[i].nitems;
    for (int l = 0; l < DAG_LANES; ++l) S.next_item[(size_t)l * a.ntasks + i] = 0;
    S.rq0[i] = -1;
    S.rq1[i] = -1;
  }
  if (i == 0) *S.ctl = DagCtl{{0, 0}, {0, 0}, 0, 0, 0, 0};
}

// The tasks without predecessors, in issue order, into their ready queues.
__global__ void dag_seed_kernel(DagArgs a) {
  DagState S = dag_state_at(a.state, a.ntasks);
  if (threadIdx.x == 0)
    for (int t = 0; t < a.ntasks; ++t)
      if (a.tasks[t].npred == 0) DevCore::publish(a.tasks, S, t);
}

// The item kinds are separate functions (not inlined into the executor loop), so that
// each is register-allocated on its own, as in its launch-per-step kernel.
template <int SPEC>
__device__ __noinline__ void dag_gemm_tile(const GemmJob& job, const GemmSeg* segs, int m0, int n0, char* smem) {
  gemm_tile_work<double, double, SPEC, DAG_WN>(job, segs, m0, n0, smem);
}

__device__ __noinline__ void dag_potrf(const DagOp& op, unsigned long long* info, char* smem) {
  potrf_block_work<64, 8>((double*)op.p0, op.i0, (double*)op.p1, op.i0, (int)op.i1, op.i2, info, threadIdx.x, smem);
}

GPR_DEV void dag_gemm_item(const DagArgs& a, const DagTask& T, int idx, char* smem) {
  int lo = T.job0, hi = T.job0 + T.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.jobs[mid].wg_begin <= idx) lo = mid; else hi = mid - 1;
  }
  const GemmJob job = a.jobs[lo];
  int m0, n0;
  job_tile(job, idx - job.wg_begin, m0, n0);
  if ((job.flags & JOB_LOWER_ONLY) && (m0 + GEMM_BM - 1 < n0)) return;
  switch (T.spec) {
    case SPEC_KK: dag_gemm_tile<SPEC_KK>(job, a.segs, m0, n0, smem); break;
    case SPEC_KM: dag_gemm_tile<SPEC_KM>(job, a.segs, m0, n0, smem); break;
    case SPEC_MM: dag_gemm_tile<SPEC_MM>(job, a.segs, m0, n0, smem); break;
    default: dag_gemm_tile<SPEC_GUARDED>(job, a.segs, m0, n0, smem); break;
  }
}

// One 64 x 64 block of a tile transpose: dst tile t = (src tile t)^T.
template <typename E>
__device__ __noinline__ void dag_transpose_item(const DagOp& op, int idx, char* smem) {
  E (*blk)[65] = reinterpret_cast<E (*)[65]>(smem);
  const int64_t b = op.i0, nbt = (b + 63) / 64, per_tile = nbt * nbt;
  const int64_t t = idx / per_tile, rem = idx % per_tile;
  const int64_t r0 = (rem / nbt) * 64, c0 = (rem % nbt) * 64;
  const E* S = (const E*)op.p1 + t * b * b;
  E* D = (E*)op.p0 + t * b * b;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 8 rows per pass
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t r = r0 + ty + 8 * q, c = c0 + tx;
    if (r < b && c < b) blk[ty + 8 * q][tx] = S[r * b + c];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t r = c0 + ty + 8 * q, c = r0 + tx;   // D[r][c] = S[c][r]
    if (r < b && c < b) D[r * b + c] = blk[tx][ty + 8 * q];
  }
}

GPR_DEV void dag_run_item(const DagArgs& a, int t, int idx, char* smem) {
  const DagTask& T = a.tasks[t];
  const int tid = threadIdx.x;
  if (T.kind == DAG_GEMM) {
    dag_gemm_item(a, T, idx, smem);
    return;
  }
  const DagOp& op = a.ops[T.op];
  switch (T.kind) {
    case DAG_POTRF:
      dag_potrf(op, a.info, smem);
      break;
    case DAG_IDENTITY:
    case DAG_ZERO_UPPER: {
      double* P = (double*)op.p0;
      const int64_t b = op.i0, total = b * b, e0 = (int64_t)idx * DAG_ELEMS_PER_ITEM;
      for (int64_t e = e0 + tid; e < e0 + DAG_ELEMS_PER_ITEM && e < total; e += DAG_THREADS) {
        const int64_t r = e / b, c = e % b;
        if (T.kind == DAG_IDENTITY) P[e] = (r == c) ? 1.0 : 0.0;
        else if (c > r) P[e] = 0.0;
      }
      break;
    }
    case DAG_COPY: {
      const uint4* S = (const uint4*)op.p1;
      uint4* D = (uint4*)op.p0;
      const int64_t n16 = op.i0 / 16, v0 = (int64_t)idx * (DAG_COPY_BYTES_PER_ITEM / 16);
      for (int64_t v = v0 + tid; v < v0 + DAG_COPY_BYTES_PER_ITEM / 16 && v < n16; v += DAG_THREADS) D[v] = S[v];
      break;
    }
    case DAG_TRANSPOSE:
      if (op.i2 == 8) dag_transpose_item<double>(op, idx, smem);
      else dag_transpose_item<float>(op, idx, smem);
      break;
    default:
      break;
  }
}

// four waves per SIMD (two workgroups per CU), as the tile-product kernels
__global__ __launch_bounds__(DAG_THREADS, 4)
void dag_kernel(DagArgs a) {
  __shared__ __align__(16) char smem[DAG_SMEM];
  __shared__ int s_task, s_idx, s_go, s_fence;
  DagState S = dag_state_at(a.state, a.ntasks);
  const int tid = threadIdx.x;
  int last = -1;
  uint64_t since = 0;
  int seen[2] = {0, 0};   // thread 0: ready-queue slots handed out before this workgroup's last acquire fence
  // the XCD this workgroup runs on (hardware register XCC_ID): its lane of each task's items
  const int lane = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % DAG_LANES);
  while (true) {
    if (tid == 0) {
      int t = 0, idx = 0, q = 0, h = 0, go = 0;
      while (true) {
        if (DevCore::try_claim(a.tasks, S, lane, t, idx, q, h)) {
          go = 1;
          break;
        }
        if (!DevCore::keep_waiting(S, last, since, a.limit)) break;
      }
      // a task published before the last acquire fence of this workgroup needs none
      int fence = 0;
      if (go && h >= seen[q]) {
        seen[0] = DagDeviceOps::load_relaxed(&S.ctl->tail[0]);
        seen[1] = DagDeviceOps::load_relaxed(&S.ctl->tail[1]);
        fence = 1;
      }
      s_task = t;
      s_idx = idx;
      s_go = go;
      s_fence = fence;
    }
    __syncthreads();
    if (!s_go) break;
    const int t = s_task, idx = s_idx;
    if (s_fence) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // no stale lines of the inputs
    dag_run_item(a, t, idx, smem);
    // every wave's stores have reached the L2 before thread 0's release (in finish) writes
    // the L2 back
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) DevCore::finish(a.tasks, a.succ, S, t);
  }
}

// Workgroups of the persistent executor that fit on the current device at once.
hipError_t dag_slots(int* slots) {
  int dev = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dag_kernel, DAG_THREADS, 0);
  if (e != hipSuccess) return e;
  *slots = (per_cu < 1 ? 1 : per_cu) * prop.multiProcessorCount;
  return hipSuccess;
}

// After the executor: a graph that gave up leaves DAG_ABORT_INFO in the pivot word.
__global__ void dag_finish_kernel(DagArgs a) {
  DagState S = dag_state_at(a.state, a.ntasks);
  if (threadIdx.x == 0 && __hip_atomic_load(&S.ctl->abort, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0)
    a.info[0] = DAG_ABORT_INFO;
}

hipError_t launch_dag(const DagTask* tasks, int ntasks, const int32_t* succ, const DagOp* ops, const GemmJob* jobs,
                      const GemmSeg* segs, int32_t* state, unsigned long long* info, double limit_s, int slots,
                      hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  if (khz <= 0) khz = 100000;   // the 100 MHz constant clock of the gfx9 family
  DagArgs a{tasks, succ, ops, jobs, segs, state, info, ntasks, (uint64_t)(limit_s * 1.0e3 * (double)khz)};
  hipLaunchKernelGGL(dag_reset_kernel, dim3((ntasks + 255) / 256), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(dag_seed_kernel, dim3(1), dim3(64), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(dag_kernel, dim3(slots < 1 ? 1 : slots), dim3(DAG_THREADS), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(dag_finish_kernel, dim3(1), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace gpr
