// The workgroup kernel of one diagonal-block factorisation; the arithmetic is in
// potrf_device.h.
#include "common.h"
#include "kernels.h"
#include "potrf_device.h"

namespace gpr {

template <int PB>
__global__ __launch_bounds__(PB * 4)
void potrf_block_kernel(double* __restrict__ A, int64_t lda, double* __restrict__ W, int64_t ldw, int jb,
                        int64_t col_base, unsigned long long* info) {
  __shared__ __align__(16) char smem[potrf_block_smem<PB>()];
  potrf_block_work<PB, 4>(A, lda, W, ldw, jb, col_base, info, threadIdx.x, smem);
}


hipError_t launch_potrf_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                              unsigned long long* info, hipStream_t st) {
  if (jb <= 0) return hipSuccess;
  if (jb > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(potrf_block_kernel<64>, dim3(1), dim3(256), 0, st, A, lda, W, ldw, jb, col_base, info);
  return hipGetLastError();
}

}  // namespace gpr
