// Small utility kernels of the factorisation: identity and zero fills, precision casts.
#include "common.h"
#include "kernels.h"

namespace gpr {

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

// dst[0..bytes) = src[0..bytes), 16 bytes per thread and step (both 16-byte aligned, bytes % 16 == 0)
__global__ void copy16_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

static int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

hipError_t launch_set_identity(double* W, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(set_identity_kernel, dim3(grid_for(b * b)), dim3(256), 0, st, W, b);
  return hipGetLastError();
}

hipError_t launch_zero_upper(double* A, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(zero_upper_kernel, dim3(grid_for(b * b)), dim3(256), 0, st, A, b);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if ((((uintptr_t)dst | (uintptr_t)src | bytes) & 15) != 0) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  const int64_t n16 = (int64_t)(bytes / 16);
  int64_t g = (n16 + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)g), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* src, float* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_f64_f32_kernel, dim3(grid_for(count)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

}  // namespace gpr
