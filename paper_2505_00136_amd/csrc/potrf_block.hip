// Factorisation and inversion of one 64 x 64 diagonal block by one workgroup in LDS.
//
// The diagonal tile of each step of the tiled factorisation (the POTRF task of
// Fig. 1) is factored by a blocked right-looking loop over 64-wide blocks (the
// orchestration issues the block steps in stream order); this kernel handles the
// diagonal block of each block step: the unblocked right-looking Cholesky (four
// threads per row) and the inverse of the factor by row operations on the identity,
// both with one barrier-separated phase per column.
#include "common.h"
#include "kernels.h"

namespace gpr {

constexpr int DB = 64;           // block edge
// Cholesky of the jb x jb block at A (in place, zero upper) and its inverse into W.
// a and w are LDS scratch of DB x (DB+1).
GPR_DEV void potrf_inv_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                             unsigned long long* info, double (*a)[DB + 1], double (*w)[DB + 1]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < DB * DB; e += 256) {
    const int i = e / DB, k = e % DB;
    a[i][k] = (i < jb && k <= i) ? A[(int64_t)i * lda + k] : 0.0;
    w[i][k] = (i == k && i < jb) ? 1.0 : 0.0;
  }
  __syncthreads();
  // right-looking unblocked Cholesky; 4 threads per row, columns strided by 4
  const int ri = tid >> 2, cq = tid & 3;
  for (int j = 0; j < jb; ++j) {
    const double dj = a[j][j];
    const double piv = sqrt(dj);
    if (tid == 0 && !(dj > 0.0)) atomicMin(info, (unsigned long long)(col_base + j + 1));
    const double inv = 1.0 / piv;
    __syncthreads();
    if (cq == 0 && ri > j && ri < jb) a[ri][j] *= inv;
    if (tid == 0) a[j][j] = piv;
    __syncthreads();
    if (ri > j && ri < jb) {
      const double lij = a[ri][j];
      for (int k = j + 1 + cq; k <= ri; k += 4) a[ri][k] -= lij * a[k][j];
    }
    __syncthreads();
  }
  // inverse by row operations on W = I: row j /= L_jj, then row i -= L_ij row j (i > j)
  for (int j = 0; j < jb; ++j) {
    const double inv = 1.0 / a[j][j];
    if (ri == j) {
      for (int c = cq; c <= j; c += 4) w[j][c] *= inv;
    }
    __syncthreads();
    if (ri > j && ri < jb) {
      const double lij = a[ri][j];
      for (int c = cq; c <= j; c += 4) w[ri][c] -= lij * w[j][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e / jb, k = e % jb;
    A[(int64_t)i * lda + k] = k <= i ? a[i][k] : 0.0;
    W[(int64_t)i * ldw + k] = k <= i ? w[i][k] : 0.0;
  }
}

__global__ __launch_bounds__(256)
void potrf_block_kernel(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                         unsigned long long* info) {
  __shared__ double a[DB][DB + 1];
  __shared__ double w[DB][DB + 1];
  potrf_inv_block(A, lda, W, ldw, jb, col_base, info, a, w);
}

hipError_t launch_potrf_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                               unsigned long long* info, hipStream_t st) {
  if (jb <= 0) return hipSuccess;
  if (jb > DB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_block_kernel, dim3(1), dim3(256), 0, st, A, lda, W, ldw, jb, col_base, info);
  return hipGetLastError();
}

}  // namespace gpr
