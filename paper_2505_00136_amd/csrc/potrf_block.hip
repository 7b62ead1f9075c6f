// Factorisation and inversion of one diagonal block (up to 64 x 64) by one workgroup.
//
// The diagonal tile of each step of the tiled factorisation (the POTRF task of
// Fig. 1) is factored by a blocked right-looking loop over 64-wide blocks (the
// orchestration issues the block steps in stream order); this kernel handles the
// diagonal block of each block step.  The block and its inverse live in registers:
// 4 threads per row, thread t owns row t/4 and every fourth column starting at t%4, of
// both L and W = L^{-1}.  One loop over the columns j does, with two barriers:
//   pivot  L_jj = sqrt(A_jj), column j of L scaled by 1/L_jj, row j of W scaled by 1/L_jj,
//   then   A_ik -= L_ij L_kj  (j < k <= i)  and  W_ic -= L_ij W_jc  (c <= j < i),
// i.e. the right-looking Cholesky fused with forward elimination of L W = I.
// Column j of L and row j of W are exchanged through two LDS vectors that are zero
// outside their ranges (L_kj for k > j, W_jc for c <= j), so the rank-1 updates run
// unmasked over all of a thread's columns: the entries they leave wrong (k > i) are
// never stored.  The next pivot column is handed over in LDS by the threads that update
// it, and column k of L keeps its unscaled value in registers until the final store
// applies 1/L_kk, so no register is indexed at run time and no global store is pending
// at any barrier.
#include "common.h"
#include "kernels.h"

namespace gpr {

// Block edge PB, PB*4 threads; thread t owns row t/4 and columns t%4 + 4q.
template <int PB>
__global__ __launch_bounds__(PB * 4)
void potrf_block_kernel(double* __restrict__ A, int64_t lda, double* __restrict__ W, int64_t ldw, int jb,
                        int64_t col_base, unsigned long long* info) {
  constexpr int PQ = PB / 4;
  // exchange vectors of step j, element k stored at [k % 4][k / 4] so that each thread's
  // operands are contiguous: exl = column j of L (zero for k <= j), exw = row j of W
  // (zero for c > j)
  __shared__ __align__(16) double exl[4][PQ];
  __shared__ __align__(16) double exw[4][PQ];
  __shared__ double nextc[PB];    // current column j of A, before scaling
  __shared__ double piv[PB];
  __shared__ double ipiv[PB];
  const int tid = threadIdx.x;
  const int i = tid >> 2, cq = tid & 3;
  double ra[PQ], rw[PQ];
#pragma unroll
  for (int q = 0; q < PQ; ++q) {
    const int k = cq + 4 * q;
    ra[q] = (i < jb && k <= i) ? A[(int64_t)i * lda + k] : 0.0;
    rw[q] = (i < jb && k == i) ? 1.0 : 0.0;
  }
  if (i < PQ) {
    exl[cq][i] = 0.0;
    exw[cq][i] = 0.0;
  }
  if (cq == 0 && i < jb) nextc[i] = ra[0];
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    if (i == j && cq == (j & 3)) {
      const double d = nextc[j];
      if (!(d > 0.0)) atomicMin(info, (unsigned long long)(col_base + j + 1));
      const double p = sqrt(d);
      piv[j] = p;
      ipiv[j] = 1.0 / p;
    }
    __syncthreads();
    const double inv = ipiv[j];
    // column j of L (its own entry k = j leaves the update vector: zero)
    if (cq == 0 && i >= j && i < jb) exl[i & 3][i >> 2] = i == j ? 0.0 : nextc[i] * inv;
    if (i == j) {                                         // row j of W is final (zero beyond j)
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        rw[q] *= inv;
        exw[cq][q] = rw[q];
      }
    }
    __syncthreads();
    if (i > j && i < jb) {
      const double li = exl[i & 3][i >> 2];
      double el[PQ], ew[PQ];
#pragma unroll
      for (int q = 0; q < PQ; q += 2) {
        const double2 vl = *reinterpret_cast<const double2*>(&exl[cq][q]);
        const double2 vw = *reinterpret_cast<const double2*>(&exw[cq][q]);
        el[q] = vl.x;
        el[q + 1] = vl.y;
        ew[q] = vw.x;
        ew[q + 1] = vw.y;
      }
      const int j1 = j + 1;
      double nv = 0.0;
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        ra[q] = fma(-li, el[q], ra[q]);
        rw[q] = fma(-li, ew[q], rw[q]);
        nv = (cq + 4 * q == j1) ? ra[q] : nv;
      }
      if (cq == (j1 & 3)) nextc[i] = nv;
    }
  }
  __syncthreads();
  // column k of L kept its unscaled value in the registers since step k
#pragma unroll
  for (int q = 0; q < PQ; ++q) {
    const int k = cq + 4 * q;
    if (i < jb && k < jb) {
      A[(int64_t)i * lda + k] = k < i ? ra[q] * ipiv[k] : (k == i ? piv[k] : 0.0);
      W[(int64_t)i * ldw + k] = k <= i ? rw[q] : 0.0;
    }
  }
}


hipError_t launch_potrf_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                              unsigned long long* info, hipStream_t st) {
  if (jb <= 0) return hipSuccess;
  if (jb > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_block_kernel<64>, dim3(1), dim3(256), 0, st, A, lda, W, ldw, jb, col_base, info);
  return hipGetLastError();
}

}  // namespace gpr
