// Bandwidth-bound kernels: matrix-vector products over tiles, partial-sum
// reductions in a fixed order (so every result is bitwise reproducible), the
// predictive-variance finish and the log marginal likelihood (Eq. 5).
#include "common.h"
#include "kernels.h"

namespace gpr {

// Sum over the 64 lanes of a wave (butterfly), the same value in every lane.
GPR_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums of two values over a 1024-thread workgroup: within each wave by shuffles, then the
// 16 wave sums in a fixed order by the first wave.  Valid in thread 0.
GPR_DEV void block_sum2(double& a, double& b) {
  __shared__ double part[2][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    part[0][wave] = a;
    part[1][wave] = b;
  }
  __syncthreads();
  if (wave == 0) {
    a = wave_sum(lane < 16 ? part[0][lane] : 0.0);
    b = wave_sum(lane < 16 ? part[1][lane] : 0.0);
  }
}

template <typename T>
__global__ __launch_bounds__(256)
void gemv_n_kernel(const T* __restrict__ A, int64_t lda, int64_t rows, int64_t cols, const double* __restrict__ x,
                   double alpha, const double* yin, double beta, double* y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const T* a = A + r * lda;
  double s0 = 0.0, s1 = 0.0;
  int64_t c = lane;
  for (; c + 64 < cols; c += 128) {
    s0 = fma((double)a[c], x[c], s0);
    s1 = fma((double)a[c + 64], x[c + 64], s1);
  }
  if (c < cols) s0 = fma((double)a[c], x[c], s0);
  const double s = wave_sum(s0 + s1);
  if (lane == 0) {
    double v = alpha * s;
    if (beta != 0.0) v += beta * yin[r];
    y[r] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256)
void gemv_t_partial_kernel(const T* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                           const double* __restrict__ x, double* __restrict__ partial, int64_t rpc, int sq) {
  const int64_t c = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int64_t rb = (int64_t)blockIdx.x * rpc;
  int64_t re = rb + rpc;
  if (re > rows) re = rows;
  if (c >= cols) return;
  double s0 = 0.0, s1 = 0.0;
  int64_t r = rb;
  if (sq) {
    for (; r + 1 < re; r += 2) {
      const double a0 = (double)A[r * lda + c], a1 = (double)A[(r + 1) * lda + c];
      s0 = fma(a0, a0, s0);
      s1 = fma(a1, a1, s1);
    }
    if (r < re) { const double a0 = (double)A[r * lda + c]; s0 = fma(a0, a0, s0); }
  } else {
    for (; r + 1 < re; r += 2) {
      s0 = fma((double)A[r * lda + c], x[r], s0);
      s1 = fma((double)A[(r + 1) * lda + c], x[r + 1], s1);
    }
    if (r < re) s0 = fma((double)A[r * lda + c], x[r], s0);
  }
  partial[(int64_t)blockIdx.x * cols + c] = s0 + s1;
}

__global__ void reduce_partials_kernel(const double* __restrict__ partial, int64_t nch, int64_t cols, double alpha,
                                       const double* yin, double beta, double* y) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t ch = 0; ch < nch; ++ch) s += partial[ch * cols + c];
  double v = alpha * s;
  if (beta != 0.0) v += beta * yin[c];
  y[c] = v;
}

__global__ void var_finish_kernel(const double* __restrict__ partial, int64_t nch, int64_t cols, HyperArg h,
                                  int add_noise, double* out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  double s = 0.0;
  for (int64_t ch = 0; ch < nch; ++ch) s += partial[ch * cols + c];
  out[c] = (add_noise ? nu + s2 : nu) - s;
}

__global__ __launch_bounds__(1024)
void nlml_kernel(const double* __restrict__ D, int64_t b, int64_t n, const double* __restrict__ y,
                 const double* __restrict__ alpha, double* out) {
  const int tid = threadIdx.x;
  double sl = 0.0, sy = 0.0;   // (padded pivots, rows n and beyond, are 1: log 0)
  for (int64_t i = tid; i < n; i += 1024) {
    const int64_t k = i / b, r = i % b;
    sl += log(D[k * b * b + r * (b + 1)]);
    sy = fma(y[i], alpha[i], sy);
  }
  block_sum2(sl, sy);
  if (tid == 0) out[0] = 0.5 * sy + sl + 0.5 * (double)n * log(2.0 * M_PI);
}

__global__ void residual_finish_kernel(const double* __restrict__ partial, int64_t nch, int64_t n, HyperArg h,
                                       const double* __restrict__ y, const double* __restrict__ alpha, double* r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  double s = 0.0;
  for (int64_t ch = 0; ch < nch; ++ch) s += partial[ch * n + i];
  r[i] = y[i] - (s + s2 * alpha[i]);
}

// The same for the symmetric products (launch_se_kmatvec_gram_sym): row i takes the row sums
// rowpart[bj][i] of the block columns bj <= i / 128, then the column sums colpart[x][i] of
// the blocks x > i / 128 below its own, in order.
__global__ void residual_finish_sym_kernel(const double* __restrict__ rowpart, const double* __restrict__ colpart,
                                           int64_t n, HyperArg h, const double* __restrict__ y,
                                           const double* __restrict__ alpha, double* r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const int64_t nb = (n + 127) / 128, bi = i / 128;
  double s = 0.0;
  for (int64_t bj = 0; bj <= bi; ++bj) s += rowpart[bj * n + i];
  for (int64_t x = bi + 1; x < nb; ++x) s += colpart[x * n + i];
  r[i] = y[i] - (s + s2 * alpha[i]);
}

__global__ void axpy_kernel(double* y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_gemv_n(const void* A, int a_f32, int64_t lda, int64_t rows, int64_t cols, const double* x,
                         double alpha, const double* yin, double beta, double* y, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (a_f32)
    hipLaunchKernelGGL(gemv_n_kernel<float>, dim3(blocks_for(rows, 4)), dim3(256), 0, st, (const float*)A, lda,
                       rows, cols, x, alpha, yin, beta, y);
  else
    hipLaunchKernelGGL(gemv_n_kernel<double>, dim3(blocks_for(rows, 4)), dim3(256), 0, st, (const double*)A,
                       lda, rows, cols, x, alpha, yin, beta, y);
  return hipGetLastError();
}

static hipError_t gemv_t_common(const void* A, int a_f32, int64_t lda, int64_t rows, int64_t cols, const double* x,
                                double* partial, int64_t rpc, int sq, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid(blocks_for(rows, (int)rpc), blocks_for(cols, 256));
  if (a_f32)
    hipLaunchKernelGGL(gemv_t_partial_kernel<float>, grid, dim3(256), 0, st, (const float*)A, lda, rows, cols, x,
                       partial, rpc, sq);
  else
    hipLaunchKernelGGL(gemv_t_partial_kernel<double>, grid, dim3(256), 0, st, (const double*)A, lda, rows, cols,
                       x, partial, rpc, sq);
  return hipGetLastError();
}

hipError_t launch_gemv_t_partial(const void* A, int a_f32, int64_t lda, int64_t rows, int64_t cols,
                                 const double* x, double* partial, int64_t rpc, hipStream_t st) {
  return gemv_t_common(A, a_f32, lda, rows, cols, x, partial, rpc, 0, st);
}

hipError_t launch_colsq_partial(const void* V, int v_f32, int64_t ld, int64_t rows, int64_t cols, double* partial,
                                int64_t rpc, hipStream_t st) {
  return gemv_t_common(V, v_f32, ld, rows, cols, nullptr, partial, rpc, 1, st);
}

hipError_t launch_reduce_partials(const double* partial, int64_t nch, int64_t cols, double alpha, const double* yin,
                                  double beta, double* y, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks_for(cols, 256)), dim3(256), 0, st, partial, nch, cols,
                     alpha, yin, beta, y);
  return hipGetLastError();
}

hipError_t launch_var_finish(const double* partial, int64_t nch, int64_t cols, HyperArg h, int add_noise,
                             double* out, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(var_finish_kernel, dim3(blocks_for(cols, 256)), dim3(256), 0, st, partial, nch, cols, h,
                     add_noise, out);
  return hipGetLastError();
}

hipError_t launch_nlml(const double* D, int64_t b, int64_t n, const double* y, const double* alpha, double* nlml,
                       hipStream_t st) {
  hipLaunchKernelGGL(nlml_kernel, dim3(1), dim3(1024), 0, st, D, b, n, y, alpha, nlml);
  return hipGetLastError();
}

hipError_t launch_residual_finish(const double* partial, int64_t nch, int64_t n, HyperArg h, const double* y,
                                  const double* alpha, double* r, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(residual_finish_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, partial, nch, n, h, y,
                     alpha, r);
  return hipGetLastError();
}

hipError_t launch_residual_finish_sym(const double* rowpart, const double* colpart, int64_t n, HyperArg h,
                                      const double* y, const double* alpha, double* r, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(residual_finish_sym_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, rowpart, colpart, n, h,
                     y, alpha, r);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}

}  // namespace gpr

namespace gpr {

__global__ __launch_bounds__(1024)
void grad_finish_kernel(const double* __restrict__ partial, int64_t nwg, HyperArg h, int64_t npadded, int t0,
                        int t1, int t2, double* grad) {
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t w = tid; w < nwg; w += 1024) {
    a += partial[w * 3 + 0];
    b += partial[w * 3 + 1];
    c += partial[w * 3 + 2];
  }
  block_sum2(a, b);
  double unused = 0.0;
  __syncthreads();   // block_sum2's wave sums are read before the next call writes them
  block_sum2(c, unused);
  if (tid == 0) {
    double ell, nu, s2;
    resolve_hyper(h, ell, nu, s2);
    // A padded row p has (K^{-1})_pp = 1 and zero elsewhere in its row and column (the
    // identity border stays exact through the factor and its inverse), zero alpha_p and
    // distance 0 to itself: it adds nu to the nu sum, 1 to the diagonal sum, 0 to the
    // length-scale sum.
    const double pad = (double)npadded;
    grad[0] = t0 ? 0.5 * a : 0.0;
    grad[1] = t1 ? 0.5 * (b - pad * nu) : 0.0;
    grad[2] = t2 ? 0.5 * s2 * (c - pad) : 0.0;
  }
}

// state = m[3], v[3], t
__global__ void adam3_kernel(double* theta, double* state, const double* grad, double lr, double b1, double b2,
                             double eps, int t0, int t1, int t2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double t = state[6] + 1.0;
  state[6] = t;
  const int tr[3] = {t0, t1, t2};
  for (int k = 0; k < 3; ++k) {
    if (!tr[k]) continue;
    const double g = grad[k];
    const double m = b1 * state[k] + (1.0 - b1) * g;
    const double v = b2 * state[3 + k] + (1.0 - b2) * g * g;
    state[k] = m;
    state[3 + k] = v;
    const double mhat = m / (1.0 - pow(b1, t));
    const double vhat = v / (1.0 - pow(b2, t));
    theta[k] -= lr * mhat / (sqrt(vhat) + eps);
  }
}

hipError_t launch_grad_finish(const double* partial, int64_t nwg, HyperArg h, int64_t npadded, int t0, int t1,
                              int t2, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(grad_finish_kernel, dim3(1), dim3(1024), 0, st, partial, nwg, h, npadded, t0, t1, t2, grad);
  return hipGetLastError();
}

hipError_t launch_adam3(double* theta, double* state, const double* grad, double lr, double b1, double b2,
                        double eps, int t0, int t1, int t2, hipStream_t st) {
  hipLaunchKernelGGL(adam3_kernel, dim3(1), dim3(64), 0, st, theta, state, grad, lr, b1, b2, eps, t0, t1, t2);
  return hipGetLastError();
}

}  // namespace gpr
