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

// dst tile t = (source tile t)^T for `count` b x b row-major tiles: one 64 x 64 block per
// workgroup, read row-wise into LDS (one padding column against bank conflicts) and
// written row-wise from its transpose, so both global sides are coalesced.  Source tile
// t is src + t b^2 (row < 0), or tile (row, t) of a region O of T x T tiles at src
// (column-major packed, index t (T-1) - t (t-1)/2 + (row - t - 1)).
template <typename E>
__global__ __launch_bounds__(256)
void transpose_tiles_kernel(const E* __restrict__ src, E* __restrict__ dst, int64_t b, int64_t nbt, int64_t T,
                            int64_t row) {
  __shared__ E blk[64][65];
  const int64_t per_tile = nbt * nbt;
  const int64_t t = blockIdx.x / per_tile, rem = blockIdx.x % per_tile;
  const int64_t r0 = (rem / nbt) * 64, c0 = (rem % nbt) * 64;
  const int64_t st = row < 0 ? t : t * (T - 1) - t * (t - 1) / 2 + (row - t - 1);
  const E* S = src + st * b * b;
  E* D = dst + t * b * b;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t r = r0 + ty + 4 * q, c = c0 + tx;
    if (r < b && c < b) blk[ty + 4 * q][tx] = S[r * b + c];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t r = c0 + ty + 4 * q, c = r0 + tx;   // D[r][c] = S[c][r]
    if (r < b && c < b) D[r * b + c] = blk[tx][ty + 4 * q];
  }
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

__global__ void copy4_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t n4) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void copy1_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Device-to-device copies are kernels (16-, 4- or 1-byte elements by alignment), never the
// runtime's copy: a runtime copy on one stream of data a kernel on another stream produced
// was observed to read stale data despite the event ordering them.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const uintptr_t al = (uintptr_t)dst | (uintptr_t)src | bytes;
  if ((al & 15) == 0) {
    const int64_t n16 = (int64_t)(bytes / 16);
    int64_t g = (n16 + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)g), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n16);
  } else if ((al & 3) == 0) {
    const int64_t n4 = (int64_t)(bytes / 4);
    int64_t g = (n4 + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(copy4_kernel, dim3((unsigned)g), dim3(256), 0, st, (const uint32_t*)src, (uint32_t*)dst, n4);
  } else {
    const int64_t n = (int64_t)bytes;
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(copy1_kernel, dim3((unsigned)g), dim3(256), 0, st, (const unsigned char*)src, (unsigned char*)dst,
                       n);
  }
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(count)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

static hipError_t transpose_common(const void* src, void* dst, int64_t b, int64_t count, int esize, int64_t T,
                                   int64_t row, hipStream_t st) {
  if (b <= 0 || count <= 0) return hipSuccess;
  const int64_t nbt = (b + 63) / 64, blocks = count * nbt * nbt;
  if (blocks > 0x7fffffff || (esize != 4 && esize != 8)) return hipErrorInvalidValue;
  if (esize == 8)
    hipLaunchKernelGGL(transpose_tiles_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (const double*)src,
                       (double*)dst, b, nbt, T, row);
  else
    hipLaunchKernelGGL(transpose_tiles_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (const float*)src,
                       (float*)dst, b, nbt, T, row);
  return hipGetLastError();
}

hipError_t launch_transpose_tiles(const void* src, void* dst, int64_t b, int64_t count, int esize, hipStream_t st) {
  return transpose_common(src, dst, b, count, esize, 0, -1, st);
}

hipError_t launch_transpose_block_row(const void* obase, int64_t T, int64_t row, void* dst, int64_t b, int esize,
                                      hipStream_t st) {
  if (row < 1 || row >= T) return row == 0 ? hipSuccess : hipErrorInvalidValue;
  return transpose_common(obase, dst, b, row, esize, T, row, st);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if ((((uintptr_t)p) | bytes) & 3) return hipErrorInvalidValue;
  const int64_t count = (int64_t)(bytes / 4);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(grid_for(count)), dim3(256), 0, st, (uint32_t*)p, count);
  return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* src, float* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_f64_f32_kernel, dim3(grid_for(count)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

}  // namespace gpr
