// Batched tile GEMM on the gfx950 matrix cores (float64 and float32 MFMA).
//
// Every dense contraction of the factorisation, the triangular inversions, the
// multi-right-hand-side forward substitution of the variance and the K^{-1}
// product of the gradient is a list of jobs C = alpha * sum_s op(A_s) op(B_s)^T + beta * Cin.
// A workgroup computes one 128x128 macro tile of one job with 2 x WN wave64s, each
// owning a 64 x (128/WN) block held as 4 x (8/WN) accumulators of the 16x16x4 MFMA:
// WN = 4 (512 threads, 64x32 per wave, four waves per SIMD) is used; WN = 2 (256
// threads, 64x64 per wave, two waves per SIMD) remains instantiable.  Operands are staged through
// double-buffered LDS in 16-deep K chunks (one barrier per chunk), the next chunk's
// global loads being in flight while the current one is multiplied.  LDS holds both
// operands k-major ([k][m]), so an MFMA fragment read by 16 consecutive lanes touches
// 16 consecutive words.
#include "common.h"
#include "gemm_device.h"
#include "kernels.h"

namespace gpr {

// Wave layout of the kernels: four waves per SIMD (WN = 4) measured 3-5% faster than two
// (WN = 2) on every operand pattern of the update, inversion and trace launches.
constexpr int WN_FACTOR = 4, WN_GRAD = 4;

// General tile products (in-tile factorisation, TRSM, solves, inversion).
template <typename T, int SPEC>
__global__ __launch_bounds__(Shape<WN_FACTOR>::THREADS, 2)
void gemm_tiles_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T, T, SPEC, WN_FACTOR>(jobs, segs, njobs);
}

// float32-stored operands multiplied in float64 (exact products): the diagonal-tile
// SYRK of the mixed-precision factorisations (KC/KC) and the full posterior covariance
// V^T V of the mixed modes (MC/MC).
template <int SPEC>
__global__ __launch_bounds__(Shape<WN_FACTOR>::THREADS, 2)
void gemm_widen_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<double, float, SPEC, WN_FACTOR>(jobs, segs, njobs);
}

// The trailing SYRK/GEMM update of a factorisation step (same code, its own symbol so
// that profiles and timings single it out).
template <typename T, int SPEC>
__global__ __launch_bounds__(Shape<WN_FACTOR>::THREADS, 2)
void gemm_update_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T, T, SPEC, WN_FACTOR>(jobs, segs, njobs);
}

// Steps of the triangular inversion L^{-1} of the gradient (same code, own symbol).
template <typename T, int SPEC>
__global__ __launch_bounds__(Shape<WN_GRAD>::THREADS, 2)
void gemm_trtri_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  gemm_tiles_body<T, T, SPEC, WN_GRAD>(jobs, segs, njobs);
}

// Gradient reduction fused into the K^{-1} = L^{-T} L^{-1} product: each job is one
// contribution X_ki^T X_kj of block row k of X = L^{-1} to the K^{-1} tile (i, j) = (aux0,
// aux1).  The macro tile never leaves registers; each element w (less alpha_r alpha_c when
// the job carries JOB_TRACE_ALPHA, once per tile) is weighted with the kernel value
// (nu exp(-u) for the squared exponential) and with its derivative with respect to
// log l (nu exp(-u) 2u = K_f r^2 / l^2; the Matern forms from u), u = r^2 / (2 l^2) read
// from the tile pair's precomputed half scaled squared distances, and the workgroup
// writes its three partial sums
// (sum w k 2u, sum w k, sum over the diagonal of w; off-diagonal tile pairs count twice,
// and a diagonal tile pair, computed on and below its diagonal only (JOB_LOWER_ONLY),
// counts its strictly-lower entries twice) to partial[blockIdx.x][0..2].
template <typename T, int SPEC>
__global__ __launch_bounds__(Shape<WN_GRAD>::THREADS, 2)
void gemm_trace_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs,
                       TraceArgs ta) {
  typedef MfmaOp<T> Op;
  typedef typename Op::acc_t acc_t;
  typedef Shape<WN_GRAD> S;
  constexpr int NJ = S::NJ;
  __shared__ __align__(16) char smem[Chunk<T>::SMEM];
  LdsBuf<T> As = reinterpret_cast<LdsBuf<T>>(smem);
  LdsBuf<T> Bs = As + 2;
  __shared__ double red[3][S::THREADS];
  GemmJob job;
  int m0, n0;
  const bool active = locate_job(jobs, njobs, job, m0, n0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = S::m0(wave), wn = S::n0(wave);
  double s_l = 0.0, s_nu = 0.0, s_s = 0.0;
  if (active) {
    acc_t acc[4][NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    gemm_mainloop<T, T, SPEC, WN_GRAD>(job, segs, m0, n0, acc, As, Bs);
    double ell, nu, s2;
    resolve_hyper(ta.h, ell, nu, s2);
    const int64_t ti = job.aux0, tj = job.aux1;
    const bool diag_tile = ti == tj;
    const bool with_alpha = job.flags & JOB_TRACE_ALPHA;
    const double* __restrict__ U = ta.u + (ti * (ti + 1) / 2 + tj) * ta.b * ta.b;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + Op::row(lane, r);
          const int col = n0 + wn + j * 16 + (lane & 15);
          // a diagonal tile pair is symmetric and computed on and below its diagonal
          // only: the strictly-lower entries count twice, the upper ones not at all
          const double wt = !diag_tile || row > col ? 2.0 : (row == col ? 1.0 : 0.0);
          if (row < job.M && col < job.N && wt != 0.0) {
            const double u = U[(int64_t)row * ta.b + col];
            double w = (double)acc[i][j][r];
            if (with_alpha) w -= ta.alpha[ti * ta.b + row] * ta.alpha[tj * ta.b + col];
            if (ta.h.kernel == KERNEL_SE) {
              const double kf = nu * exp(-u);
              s_l = fma(wt * w * kf, 2.0 * u, s_l);
              s_nu = fma(wt * w, kf, s_nu);
            } else {
              double kf, dl;
              matern_and_dlogl(ta.h.kernel, u, nu, kf, dl);
              s_l = fma(wt * w, dl, s_l);
              s_nu = fma(wt * w, kf, s_nu);
            }
            if (diag_tile && row == col) s_s += w;
          }
        }
  }
  red[0][tid] = s_l;
  red[1][tid] = s_nu;
  red[2][tid] = s_s;
  __syncthreads();
  for (int s = S::THREADS / 2; s > 0; s >>= 1) {
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

// Host: the specialised main loop a launch may use (SPEC_GUARDED if any job or segment
// needs guards or the segments mix operand modes).  esize: bytes per stored operand element;
// bk: chunk depth of the launch's product type.
int gemm_launch_spec(const GemmJob* jobs, int njobs, const GemmSeg* segs, int esize, int bk) {
  int spec = -2;
  auto aligned = [](const void* p, int64_t ld, int es) {
    return (((uintptr_t)p) & 15) == 0 && (ld * es) % 16 == 0;
  };
  for (int j = 0; j < njobs; ++j) {
    const GemmJob& J = jobs[j];
    if (J.M % GEMM_BM != 0 || J.N % GEMM_BN != 0) return SPEC_GUARDED;
    for (int q = J.seg0; q < J.seg0 + J.nseg; ++q) {
      const GemmSeg& S = segs[q];
      if (S.K % bk != 0 || !aligned(S.A, S.lda, esize) || !aligned(S.B, S.ldb, esize)) return SPEC_GUARDED;
      const int sp = S.modeA * 2 + S.modeB;
      if (spec == -2) spec = sp;
      else if (spec != sp) return SPEC_GUARDED;
    }
  }
  return spec < 0 ? SPEC_GUARDED : spec;
}

#define GPR_GEMM_LAUNCH(kern) \
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(Shape<WN_FACTOR>::THREADS), 0, st, jobs, segs, njobs)
#define GPR_GRAD_LAUNCH(kern) \
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(Shape<WN_GRAD>::THREADS), 0, st, jobs, segs, njobs)

template <typename T>
hipError_t launch_tiles_t(const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int spec, hipStream_t st) {
  if (spec == SPEC_KK) GPR_GEMM_LAUNCH((gemm_tiles_kernel<T, SPEC_KK>));
  else if (spec == SPEC_KM) GPR_GEMM_LAUNCH((gemm_tiles_kernel<T, SPEC_KM>));
  else if (spec == SPEC_MM) GPR_GEMM_LAUNCH((gemm_tiles_kernel<T, SPEC_MM>));
  else GPR_GEMM_LAUNCH((gemm_tiles_kernel<T, SPEC_GUARDED>));
  return hipGetLastError();
}

hipError_t launch_gemm(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int kind, int spec,
                       hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (kind == GEMM_KIND_BF16X3_T256 || kind == GEMM_KIND_BF16X6_T256)
    return launch_gemm_bf16_t256(gemm_kind_nprod(kind), jobs, segs, njobs, nwg, st);
  if (kind == GEMM_KIND_BF16X3_TRTRI_T256 || kind == GEMM_KIND_BF16X6_TRTRI_T256)
    return launch_gemm_bf16_trtri_t256(gemm_kind_nprod(kind), jobs, segs, njobs, nwg, st);
  if (gemm_kind_solve(kind)) return launch_gemm_bf16_solve_t256(gemm_kind_nprod(kind), jobs, segs, njobs, nwg, st);
  if (kind == GEMM_KIND_BF16X3 || kind == GEMM_KIND_BF16X6)
    return launch_gemm_bf16(gemm_kind_nprod(kind), jobs, segs, njobs, nwg, st);
  if (gemm_kind_trace(kind)) return hipErrorInvalidValue;   // launched by launch_gemm_trace
  if (kind == GEMM_KIND_WIDEN) {
    if (spec == SPEC_KK) GPR_GEMM_LAUNCH((gemm_widen_kernel<SPEC_KK>));
    else if (spec == SPEC_MM) GPR_GEMM_LAUNCH((gemm_widen_kernel<SPEC_MM>));
    else GPR_GEMM_LAUNCH((gemm_widen_kernel<SPEC_GUARDED>));
  } else if (kind == GEMM_KIND_TRTRI) {
    if (prec_f32) {
      if (spec == SPEC_MM) GPR_GRAD_LAUNCH((gemm_trtri_kernel<float, SPEC_MM>));
      else if (spec == SPEC_KM) GPR_GRAD_LAUNCH((gemm_trtri_kernel<float, SPEC_KM>));
      else GPR_GRAD_LAUNCH((gemm_trtri_kernel<float, SPEC_GUARDED>));
    } else {
      if (spec == SPEC_MM) GPR_GRAD_LAUNCH((gemm_trtri_kernel<double, SPEC_MM>));
      else if (spec == SPEC_KM) GPR_GRAD_LAUNCH((gemm_trtri_kernel<double, SPEC_KM>));
      else GPR_GRAD_LAUNCH((gemm_trtri_kernel<double, SPEC_GUARDED>));
    }
  } else if (kind == GEMM_KIND_UPDATE) {
    if (prec_f32) {
      if (spec == SPEC_MM) GPR_GEMM_LAUNCH((gemm_update_kernel<float, SPEC_MM>));
      else GPR_GEMM_LAUNCH((gemm_update_kernel<float, SPEC_GUARDED>));
    } else {
      if (spec == SPEC_MM) GPR_GEMM_LAUNCH((gemm_update_kernel<double, SPEC_MM>));
      else GPR_GEMM_LAUNCH((gemm_update_kernel<double, SPEC_GUARDED>));
    }
  } else {
    return prec_f32 ? launch_tiles_t<float>(jobs, segs, njobs, nwg, spec, st)
                    : launch_tiles_t<double>(jobs, segs, njobs, nwg, spec, st);
  }
  return hipGetLastError();
}
#undef GPR_GEMM_LAUNCH
#undef GPR_GRAD_LAUNCH

hipError_t launch_gemm_trace(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int spec,
                             const TraceArgs& ta, hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  const dim3 g(nwg), blk(Shape<WN_GRAD>::THREADS);
  if (prec_f32) {
    if (spec == SPEC_MM) hipLaunchKernelGGL((gemm_trace_kernel<float, SPEC_MM>), g, blk, 0, st, jobs, segs, njobs, ta);
    else hipLaunchKernelGGL((gemm_trace_kernel<float, SPEC_GUARDED>), g, blk, 0, st, jobs, segs, njobs, ta);
  } else {
    if (spec == SPEC_MM) hipLaunchKernelGGL((gemm_trace_kernel<double, SPEC_MM>), g, blk, 0, st, jobs, segs, njobs, ta);
    else hipLaunchKernelGGL((gemm_trace_kernel<double, SPEC_GUARDED>), g, blk, 0, st, jobs, segs, njobs, ta);
  }
  return hipGetLastError();
}

}  // namespace gpr
