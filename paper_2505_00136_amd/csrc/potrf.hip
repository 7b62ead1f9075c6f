// Diagonal-block Cholesky with its triangular inverse, and small utility kernels.
//
// The diagonal tile of each step of the tiled factorisation (the POTRF task of
// Fig. 1) is factored by a blocked right-looking loop whose jb <= 64 diagonal
// blocks are handled here by one workgroup entirely in LDS: the unblocked
// Cholesky of the block, then the inverse of its lower factor by column-wise
// forward substitution (each thread owns one column, so no barriers).
#include "common.h"
#include "kernels.h"

namespace gpr {

constexpr int PB = 64;

__global__ __launch_bounds__(256)
void potrf_block_kernel(double* __restrict__ A, int64_t lda, double* __restrict__ W, int64_t ldw, int jb,
                        int64_t col_base, unsigned long long* info) {
  __shared__ double a[PB][PB + 1];
  __shared__ double w[PB][PB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < jb * jb; idx += 256) {
    const int i = idx / jb, k = idx % jb;
    a[i][k] = (k <= i) ? A[(int64_t)i * lda + k] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    const double dj = a[j][j];
    const double piv = sqrt(dj);
    if (!(dj > 0.0) && tid == 0) atomicMin(info, (unsigned long long)(col_base + j + 1));
    __syncthreads();
    const double inv = 1.0 / piv;
    if (tid == 0) a[j][j] = piv;
    for (int i = j + 1 + tid; i < jb; i += 256) a[i][j] *= inv;
    __syncthreads();
    const int rem = jb - j - 1;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int ii = idx / rem, kk = idx % rem;
      if (kk <= ii) a[j + 1 + ii][j + 1 + kk] -= a[j + 1 + ii][j] * a[j + 1 + kk][j];
    }
    __syncthreads();
  }
  if (tid < jb) {
    const int c = tid;
    for (int i = 0; i < c; ++i) w[i][c] = 0.0;
    for (int i = c; i < jb; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= a[i][k] * w[k][c];
      w[i][c] = s / a[i][i];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < jb * jb; idx += 256) {
    const int i = idx / jb, k = idx % jb;
    A[(int64_t)i * lda + k] = a[i][k];
    W[(int64_t)i * ldw + k] = w[i][k];
  }
}

__global__ void set_identity_kernel(double* W, int64_t b) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / b, k = idx % b;
    W[idx] = (i == k) ? 1.0 : 0.0;
  }
}

__global__ void zero_upper_kernel(double* A, int64_t b) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / b, k = idx % b;
    if (k > i) A[idx] = 0.0;
  }
}

__global__ void convert_f64_f32_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t count) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * blockDim.x)
    d[idx] = (float)s[idx];
}

static int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

hipError_t launch_potrf_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                              unsigned long long* info, hipStream_t st) {
  if (jb <= 0) return hipSuccess;
  if (jb > PB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_block_kernel, dim3(1), dim3(256), 0, st, A, lda, W, ldw, jb, col_base, info);
  return hipGetLastError();
}

hipError_t launch_set_identity(double* W, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(set_identity_kernel, dim3(grid_for(b * b)), dim3(256), 0, st, W, b);
  return hipGetLastError();
}

hipError_t launch_zero_upper(double* A, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(zero_upper_kernel, dim3(grid_for(b * b)), dim3(256), 0, st, A, b);
  return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* src, float* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_f64_f32_kernel, dim3(grid_for(count)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

}  // namespace gpr
