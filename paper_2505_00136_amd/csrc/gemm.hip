// Batched tile GEMM on the gfx950 matrix cores (float64 and float32 MFMA).
//
// Every dense contraction of the factorisation, the triangular inversions, the
// multi-right-hand-side forward substitution of the variance and the K^{-1}
// product of the gradient is a list of jobs C = alpha * sum_s op(A_s) op(B_s)^T + beta * Cin.
// A 256-thread workgroup computes one 128x128 macro tile of one job; its four
// wave64s each own a 64x64 quadrant held as 4x4 accumulators of the 16x16x4
// MFMA.  Operands are staged through double-buffered LDS in 16-deep K chunks
// (one barrier per chunk), the next chunk's global loads being in flight while
// the current one is multiplied.  LDS holds both operands k-major ([k][m]), so
// an MFMA fragment read by 16 consecutive lanes touches 16 consecutive words.
#include "common.h"
#include "kernels.h"

namespace gpr {

template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
  typedef v4d acc_t;
  static GPR_DEV acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // f64 16x16x4 output: lane l, register r holds row (l/16) + 4r, column l%16
  static GPR_DEV int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MfmaOp<float> {
  typedef v4f acc_t;
  static GPR_DEV acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // f32 16x16x4 output: lane l, register r holds row 4(l/16) + r, column l%16
  static GPR_DEV int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int LDS_PAD = 4;
// double-buffered A and B chunks of the widest element type (float64)
constexpr int SMEM_BYTES = 2 * 2 * GEMM_BK * (GEMM_BM + LDS_PAD) * 8;

template <typename T>
GPR_DEV void seg_krange(const GemmSeg& s, int m0, int n0, int& kb, int& ke) {
  kb = 0;
  ke = s.K;
  if (s.tri & A_LOWER) ke = min(ke, m0 + GEMM_BM);
  if (s.tri & B_LOWER) ke = min(ke, n0 + GEMM_BN);
  if (s.tri & A_UPPER) kb = max(kb, m0);
  if (s.tri & B_UPPER) kb = max(kb, n0);
  kb = (kb / GEMM_BK) * GEMM_BK;
}

// Loads this thread's share of a 128 x 16 operand chunk into registers (zero outside
// [0,lim) x [k0,kend)).  When the whole chunk is in range and the rows are 16-byte
// aligned (a uniform test), the loads are unguarded 16-byte vector loads; otherwise
// every element is guarded.
template <typename T>
GPR_DEV void load_chunk(const T* __restrict__ P, int64_t ld, int mode, int base, int lim,
                        int k0, int kend, int tid, T (&r)[8]) {
  constexpr int VEC = 16 / sizeof(T);   // elements per 16-byte load
  const bool aligned = ((((uintptr_t)P) & 15) == 0) && (ld % VEC == 0);
  if (mode == MODE_KC) {
    const int kk = k0 + (tid & 7) * 2;
    if (aligned && base + GEMM_BM <= lim && k0 + GEMM_BK <= kend && (VEC == 2)) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int row = base + (tid >> 3) + 32 * p;
        const T* q = P + (int64_t)row * ld + kk;
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 v = *reinterpret_cast<const v2*>(q);
        r[2 * p] = v[0];
        r[2 * p + 1] = v[1];
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int row = base + (tid >> 3) + 32 * p;
      const bool rok = row < lim;
      const T* q = P + (int64_t)row * ld + kk;
      r[2 * p] = (rok && kk < kend) ? q[0] : T(0);
      r[2 * p + 1] = (rok && kk + 1 < kend) ? q[1] : T(0);
    }
  } else {
    const int k = k0 + (tid >> 4);
    const int r0 = base + (tid & 15) * 8;
    const T* q = P + (int64_t)k * ld + r0;
    if (aligned && base + GEMM_BM <= lim && k0 + GEMM_BK <= kend) {
      typedef T vv __attribute__((ext_vector_type(VEC)));
#pragma unroll
      for (int e = 0; e < 8; e += VEC) {
        const vv v = *reinterpret_cast<const vv*>(q + e);
#pragma unroll
        for (int x = 0; x < VEC; ++x) r[e + x] = v[x];
      }
      return;
    }
    const bool kok = k < kend;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (kok && r0 + e < lim) ? q[e] : T(0);
  }
}

template <typename T, typename TL>
GPR_DEV void store_chunk(T (*S)[GEMM_BM + LDS_PAD], int mode, int tid, const TL (&r)[8]) {
  if (mode == MODE_KC) {
    const int kk = (tid & 7) * 2;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int row = (tid >> 3) + 32 * p;
      S[kk][row] = (T)r[2 * p];
      S[kk + 1][row] = (T)r[2 * p + 1];
    }
  } else {
    const int k = tid >> 4;
    const int r0 = (tid & 15) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[k][r0 + e] = (T)r[e];
  }
}

// Finds this workgroup's job and macro tile; returns false when the tile lies above
// the diagonal of a lower-only job.
GPR_DEV bool locate_job(const GemmJob* __restrict__ jobs, int njobs, GemmJob& job, int& m0, int& n0) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_begin <= bid) lo = mid; else hi = mid - 1;
  }
  job = jobs[lo];
  const int t = bid - job.wg_begin;
  m0 = (t / job.tiles_n) * GEMM_BM;
  n0 = (t % job.tiles_n) * GEMM_BN;
  return !((job.flags & JOB_LOWER_ONLY) && (m0 + GEMM_BM - 1 < n0));
}

// acc += sum over the job's segments of the 128 x 128 macro tile at (m0, n0); operands are
// stored as TL and multiplied as T (float operands may be widened to float64 products).
template <typename T, typename TL = T>
GPR_DEV void gemm_mainloop(const GemmJob& job, const GemmSeg* __restrict__ segs, int m0, int n0,
                           typename MfmaOp<T>::acc_t (&acc)[4][4], T (*As)[GEMM_BK][GEMM_BM + LDS_PAD],
                           T (*Bs)[GEMM_BK][GEMM_BN + LDS_PAD]) {
  typedef MfmaOp<T> Op;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int send = job.seg0 + job.nseg;
  int cs = job.seg0, ck0 = 0, cke = 0;
  for (; cs < send; ++cs) {
    seg_krange<T>(segs[cs], m0, n0, ck0, cke);
    if (ck0 < cke) break;
  }
  if (cs >= send) return;
  TL ra[8], rb[8];
  {
    const GemmSeg& s = segs[cs];
    load_chunk<TL>((const TL*)s.A, s.lda, s.modeA, m0, job.M, ck0, cke, tid, ra);
    load_chunk<TL>((const TL*)s.B, s.ldb, s.modeB, n0, job.N, ck0, cke, tid, rb);
    store_chunk<T, TL>(As[0], s.modeA, tid, ra);
    store_chunk<T, TL>(Bs[0], s.modeB, tid, rb);
  }
  __syncthreads();
  int buf = 0;
  while (true) {
    int ns = cs, nk0 = ck0 + GEMM_BK, nke = cke;
    if (nk0 >= cke) {
      for (ns = cs + 1; ns < send; ++ns) {
        seg_krange<T>(segs[ns], m0, n0, nk0, nke);
        if (nk0 < nke) break;
      }
    }
    const bool more = ns < send;
    int nmodeA = 0, nmodeB = 0;
    if (more) {
      const GemmSeg& s = segs[ns];
      nmodeA = s.modeA;
      nmodeB = s.modeB;
      load_chunk<TL>((const TL*)s.A, s.lda, s.modeA, m0, job.M, nk0, nke, tid, ra);
      load_chunk<TL>((const TL*)s.B, s.ldb, s.modeB, n0, job.N, nk0, nke, tid, rb);
    }
#pragma unroll
    for (int kq = 0; kq < GEMM_BK / 4; ++kq) {
      const int kr = kq * 4 + (lane >> 4);
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Op::mma(a[i], b[j], acc[i][j]);
    }
    if (!more) break;
    store_chunk<T, TL>(As[buf ^ 1], nmodeA, tid, ra);
    store_chunk<T, TL>(Bs[buf ^ 1], nmodeB, tid, rb);
    __syncthreads();
    buf ^= 1;
    cs = ns;
    ck0 = nk0;
    cke = nke;
  }
}

template <typename T, typename TL = T>
GPR_DEV void gemm_tiles_body(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  typedef MfmaOp<T> Op;
  typedef typename Op::acc_t acc_t;
  __shared__ __align__(16) char smem[SMEM_BYTES];
  T (*As)[GEMM_BK][GEMM_BM + LDS_PAD] = reinterpret_cast<T (*)[GEMM_BK][GEMM_BM + LDS_PAD]>(smem);
  T (*Bs)[GEMM_BK][GEMM_BN + LDS_PAD] = As + 2;
  GemmJob job;
  int m0, n0;
  if (!locate_job(jobs, njobs, job, m0, n0)) return;
  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  gemm_mainloop<T, TL>(job, segs, m0, n0, acc, As, Bs);

  // epilogue: C = alpha * acc + beta * Cin
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const bool c32 = job.flags & JOB_C_F32;
  const double alpha = job.alpha, beta = job.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + Op::row(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < job.M && col < job.N) {
          double v = alpha * (double)acc[i][j][r];
          if (c32) {
            if (beta != 0.0) v += beta * (double)((const float*)job.Cin)[(int64_t)row * job.ldcin + col];
            ((float*)job.C)[(int64_t)row * job.ldc + col] = (float)v;
          } else {
            if (beta != 0.0) v += beta * ((const double*)job.Cin)[(int64_t)row * job.ldcin + col];
            ((double*)job.C)[(int64_t)row * job.ldc + col] = v;
          }
        }
      }
}

// General tile products (in-tile factorisation, TRSM, solves, inversion).
template <typename T>
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_tiles_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T>(jobs, segs, njobs);
}

// float32-stored operands multiplied in float64 (exact products): the diagonal-tile
// SYRK of the mixed-precision factorisations.
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_widen_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<double, float>(jobs, segs, njobs);
}

// The trailing SYRK/GEMM update of a factorisation step (same code, its own symbol so
// that profiles and timings single it out).
template <typename T>
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_update_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T>(jobs, segs, njobs);
}

// Steps of the triangular inversion L^{-1} of the gradient (same code, own symbol).
template <typename T>
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_trtri_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T>(jobs, segs, njobs);
}

// Gradient reduction fused into the K^{-1} = L^{-T} L^{-1} product: each job is one
// contribution X_ki^T X_kj of block row k of X = L^{-1} to the K^{-1} tile (i, j) = (aux0,
// aux1).  The macro tile never leaves registers; each element w (less alpha_r alpha_c when
// the job carries JOB_TRACE_ALPHA, once per tile) is weighted with the kernel value
// nu exp(-u) and with 2u = r^2 / l^2, u read from the tile pair's precomputed half scaled
// squared distances, and the workgroup writes its three partial sums
// (sum w k 2u, sum w k, sum over the diagonal of w; off-diagonal tile pairs count twice)
// to partial[blockIdx.x][0..2].
template <typename T>
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_trace_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs,
                       TraceArgs ta) {
  typedef MfmaOp<T> Op;
  typedef typename Op::acc_t acc_t;
  __shared__ __align__(16) char smem[SMEM_BYTES];
  T (*As)[GEMM_BK][GEMM_BM + LDS_PAD] = reinterpret_cast<T (*)[GEMM_BK][GEMM_BM + LDS_PAD]>(smem);
  T (*Bs)[GEMM_BK][GEMM_BN + LDS_PAD] = As + 2;
  __shared__ double red[3][GEMM_THREADS];
  GemmJob job;
  int m0, n0;
  const bool active = locate_job(jobs, njobs, job, m0, n0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  double s_l = 0.0, s_nu = 0.0, s_s = 0.0;
  if (active) {
    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    gemm_mainloop<T>(job, segs, m0, n0, acc, As, Bs);
    double ell, nu, s2;
    resolve_hyper(ta.h, ell, nu, s2);
    const int64_t ti = job.aux0, tj = job.aux1;
    const double wt = (ti == tj) ? 1.0 : 2.0;
    const bool with_alpha = job.flags & JOB_TRACE_ALPHA;
    const double* __restrict__ U = ta.u + (ti * (ti + 1) / 2 + tj) * ta.b * ta.b;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + Op::row(lane, r);
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < job.M && col < job.N) {
            const double u = U[(int64_t)row * ta.b + col];
            double w = (double)acc[i][j][r];
            if (with_alpha) w -= ta.alpha[ti * ta.b + row] * ta.alpha[tj * ta.b + col];
            const double kf = nu * exp(-u);
            s_l = fma(wt * w * kf, 2.0 * u, s_l);
            s_nu = fma(wt * w, kf, s_nu);
            if (ti == tj && row == col) s_s += w;
          }
        }
  }
  red[0][tid] = s_l;
  red[1][tid] = s_nu;
  red[2][tid] = s_s;
  __syncthreads();
  for (int s = GEMM_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
      red[2][tid] += red[2][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* o = ta.partial + (int64_t)blockIdx.x * 3;
    o[0] = red[0][0];
    o[1] = red[1][0];
    o[2] = red[2][0];
  }
}

hipError_t launch_gemm(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int kind,
                       hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (kind == GEMM_KIND_BF16X3 || kind == GEMM_KIND_BF16X6)
    return launch_gemm_bf16(kind == GEMM_KIND_BF16X6 ? 6 : 3, jobs, segs, njobs, nwg, st);
  if (kind == GEMM_KIND_WIDEN) {
    hipLaunchKernelGGL(gemm_widen_kernel, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
    return hipGetLastError();
  }
  if (kind == GEMM_KIND_TRTRI) {
    if (prec_f32)
      hipLaunchKernelGGL(gemm_trtri_kernel<float>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
    else
      hipLaunchKernelGGL(gemm_trtri_kernel<double>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
    return hipGetLastError();
  }
  if (kind == GEMM_KIND_TRACE) return hipErrorInvalidValue;   // launched by launch_gemm_trace
  if (kind == GEMM_KIND_UPDATE) {
    if (prec_f32)
      hipLaunchKernelGGL(gemm_update_kernel<float>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
    else
      hipLaunchKernelGGL(gemm_update_kernel<double>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
  } else {
    if (prec_f32)
      hipLaunchKernelGGL(gemm_tiles_kernel<float>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
    else
      hipLaunchKernelGGL(gemm_tiles_kernel<double>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
  }
  return hipGetLastError();
}

}  // namespace gpr

namespace gpr {
hipError_t launch_gemm_trace(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                             const TraceArgs& ta, hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (prec_f32)
    hipLaunchKernelGGL(gemm_trace_kernel<float>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs, ta);
  else
    hipLaunchKernelGGL(gemm_trace_kernel<double>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs, ta);
  return hipGetLastError();
}
}  // namespace gpr
