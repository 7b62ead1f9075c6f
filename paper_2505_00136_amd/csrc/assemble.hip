// Covariance blocks (Eq. 2, or a Matern kernel), computed from LDS-staged feature blocks.
//
// A 256-thread workgroup produces a 64 x 64 block of kernel values: the 64 row
// points and the 64 column points are staged into LDS 32 features at a time
// (coalesced row reads, stored feature-major), each thread accumulates the
// squared distances of its 4 x 4 outputs with explicit differences in float64,
// and the block is written with 16 consecutive threads covering 64 consecutive
// columns.  The same block routine serves the tiled training covariance, the
// dense cross- and test-covariances, and the fused kernel-vector products of
// the posterior mean (Eq. 3) and of the refinement residual.
#include "common.h"
#include "kernels.h"

namespace gpr {

constexpr int KB = 64;   // block edge
constexpr int DC = 32;   // features per LDS stage

// r2[4][4] for rows ra0.. (global indices into A, `rows` valid) and cols cb0.. of B
GPR_DEV void sqdist_block(const double* __restrict__ A, int64_t rows, int64_t ra0, const double* __restrict__ B,
                          int64_t cols, int64_t cb0, int64_t d, double (*za)[KB], double (*zb)[KB],
                          double r2[4][4]) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) r2[i][j] = 0.0;
  const int lr = tid >> 2;          // 0..63 point within the block
  const int lf = (tid & 3) * 8;     // 8 features per thread
  for (int64_t f0 = 0; f0 < d; f0 += DC) {
    __syncthreads();
    {
      const int64_t ga = ra0 + lr, gb = cb0 + lr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t f = f0 + lf + e;
        za[lf + e][lr] = (ga < rows && f < d) ? A[ga * d + f] : 0.0;
        zb[lf + e][lr] = (gb < cols && f < d) ? B[gb * d + f] : 0.0;
      }
    }
    __syncthreads();
    const int fc = (int)((d - f0) < DC ? (d - f0) : DC);
    for (int f = 0; f < fc; ++f) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = za[f][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = zb[f][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double df = a[i] - b[j];
          r2[i][j] = fma(df, df, r2[i][j]);
        }
    }
  }
}

// One-dimensional grid over (tile pair, 64 x 64 block of the tile), pair-major.
__global__ __launch_bounds__(256)
void assemble_tiles_kernel(const double* __restrict__ Z, int64_t d, HyperArg h, TileLayout L, void* K) {
  __shared__ double za[DC][KB];
  __shared__ double zb[DC][KB];
  const int64_t nbt = (L.b + KB - 1) / KB;
  const int64_t y = (int64_t)blockIdx.x / (nbt * nbt), blk = (int64_t)blockIdx.x % (nbt * nbt);
  int64_t ti, tj;
  pair_of(y, ti, tj);
  const int64_t br = blk / nbt, bc = blk % nbt;
  const int64_t r0 = br * KB, c0 = bc * KB;   // within the tile
  double r2[4][4];
  const int64_t ri = L.rows_of(ti), rj = L.rows_of(tj);   // real (unpadded) rows of the two tiles
  sqdist_block(Z + ti * L.b * d, ri, r0, Z + tj * L.b * d, rj, c0, d, za, zb, r2);
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const CovFn kf(h.kernel, ell, nu);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const bool diag = ti == tj;
  double* Dt = diag ? L.diag(K, ti) : nullptr;
  void* Ot = diag ? nullptr : L.off(K, ti, tj);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty * 4 + i;
    if (r >= L.b) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = c0 + tx * 4 + j;
      if (c >= L.b) continue;
      double v = kf(r2[i][j]);
      if (r >= ri || c >= rj) v = 0.0;   // padding: identity block, zero border
      if (diag) {
        if (r == c) v = r < ri ? v + s2 : 1.0;
        Dt[r * L.b + c] = v;
      } else if (L.esize == 8) {
        ((double*)Ot)[r * L.b + c] = v;
      } else {
        ((float*)Ot)[r * L.b + c] = (float)v;
      }
    }
  }
}

// u = r^2 / (2 l^2) for every lower tile pair, float64, pair tiles packed row-major
// (pair y = ti (ti+1)/2 + tj at U + y b^2): the squared distances of the gradient
// reduction, regenerated from Z once per gradient call.
__global__ __launch_bounds__(256)
void halfdist_tiles_kernel(const double* __restrict__ Z, int64_t n, int64_t d, HyperArg h, int64_t b,
                           double* __restrict__ U) {
  __shared__ double za[DC][KB];
  __shared__ double zb[DC][KB];
  const int64_t nbt = (b + KB - 1) / KB;
  const int64_t y = (int64_t)blockIdx.x / (nbt * nbt), blk = (int64_t)blockIdx.x % (nbt * nbt);
  int64_t ti, tj;
  pair_of(y, ti, tj);
  const int64_t r0 = (blk / nbt) * KB, c0 = (blk % nbt) * KB;
  double r2[4][4];
  // padded rows (n..Tb-1) read as zero features; the reduction gives them zero weight
  const int64_t ri = n - ti * b < b ? n - ti * b : b, rj = n - tj * b < b ? n - tj * b : b;
  sqdist_block(Z + ti * b * d, ri, r0, Z + tj * b * d, rj, c0, d, za, zb, r2);
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const double g = 0.5 / (ell * ell);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double* Ut = U + y * b * b;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty * 4 + i;
    if (r >= b) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = c0 + tx * 4 + j;
      if (c < b) Ut[r * b + c] = g * r2[i][j];
    }
  }
}

__global__ __launch_bounds__(256)
void assemble_dense_kernel(const double* __restrict__ A, int64_t rows, const double* __restrict__ B, int64_t cols,
                           int64_t d, HyperArg h, int add_diag, void* out, int64_t ld, int out_f32) {
  __shared__ double za[DC][KB];
  __shared__ double zb[DC][KB];
  const int64_t r0 = (int64_t)blockIdx.y * KB, c0 = (int64_t)blockIdx.x * KB;
  double r2[4][4];
  sqdist_block(A, rows, r0, B, cols, c0, d, za, zb, r2);
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const CovFn kf(h.kernel, ell, nu);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty * 4 + i;
    if (r >= rows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = c0 + tx * 4 + j;
      if (c >= cols) continue;
      double v = kf(r2[i][j]);
      if (add_diag && r == c) v += s2;
      if (out_f32) ((float*)out)[r * ld + c] = (float)v;
      else ((double*)out)[r * ld + c] = v;
    }
  }
}

// partial[chunk][i] = sum_{j in chunk} k(A_i, B_j) v_j ; grid (row blocks, chunks)
__global__ __launch_bounds__(256)
void kmatvec_partial_kernel(const double* __restrict__ A, int64_t rows, const double* __restrict__ B, int64_t cols,
                            int64_t d, HyperArg h, const double* __restrict__ v, double* __restrict__ partial,
                            int64_t chunk_cols) {
  __shared__ double za[DC][KB];
  __shared__ double zb[DC][KB];
  __shared__ double red[KB][17];
  const int64_t r0 = (int64_t)blockIdx.x * KB;
  const int64_t cbeg = (int64_t)blockIdx.y * chunk_cols;
  int64_t cend = cbeg + chunk_cols;
  if (cend > cols) cend = cols;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const CovFn kf(h.kernel, ell, nu);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = cbeg; c0 < cend; c0 += KB) {
    double r2[4][4];
    sqdist_block(A, rows, r0, B, cend, c0, d, za, zb, r2);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = c0 + tx * 4 + j;
      const double vc = (c < cend) ? v[c] : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = fma(kf(r2[i][j]), vc, acc[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[ty * 4 + i][tx] = acc[i];
  __syncthreads();
  if (tid < KB) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += red[tid][q];
    const int64_t r = r0 + tid;
    if (r < rows) partial[(int64_t)blockIdx.y * rows + r] = s;
  }
}

hipError_t launch_assemble_tiles(const double* Z, int64_t d, HyperArg h, const TileLayout& L, void* K,
                                 hipStream_t st) {
  if (L.T == 0) return hipSuccess;
  if (L.n <= (L.T - 1) * L.b || L.n > L.npad()) return hipErrorInvalidValue;
  // the squared exponential forms its distances on the matrix cores (gram.hip)
  if (h.kernel == KERNEL_SE) return launch_se_tiles_gram(Z, d, h, L, K, nullptr, st);
  const int64_t nbt = (L.b + KB - 1) / KB;
  const int64_t blocks = nbt * nbt * (L.T * (L.T + 1) / 2);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(assemble_tiles_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Z, d, h, L, K);
  return hipGetLastError();
}

hipError_t launch_halfdist_tiles(const double* Z, int64_t n, int64_t d, HyperArg h, int64_t b, int64_t T, double* U,
                                 hipStream_t st) {
  if (T == 0) return hipSuccess;
  const int64_t nbt = (b + KB - 1) / KB;
  const int64_t blocks = nbt * nbt * (T * (T + 1) / 2);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (n <= (T - 1) * b || n > T * b) return hipErrorInvalidValue;
  if (h.kernel == KERNEL_SE) {
    TileLayout L{n, b, T, 8};
    return launch_se_tiles_gram(Z, d, h, L, nullptr, U, st);
  }
  hipLaunchKernelGGL(halfdist_tiles_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Z, n, d, h, b, U);
  return hipGetLastError();
}

hipError_t launch_assemble_dense(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                 HyperArg h, int add_diag, void* out, int64_t ld, int out_f32,
                                 hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((unsigned)((cols + KB - 1) / KB), (unsigned)((rows + KB - 1) / KB));
  hipLaunchKernelGGL(assemble_dense_kernel, grid, dim3(256), 0, st, A, rows, B, cols, d, h, add_diag, out, ld,
                     out_f32);
  return hipGetLastError();
}

hipError_t launch_kmatvec_partial(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                  HyperArg h, const double* v, double* partial, int64_t chunk_cols,
                                  hipStream_t st) {
  if (rows == 0) return hipSuccess;
  const int64_t nch = cols == 0 ? 0 : (cols + chunk_cols - 1) / chunk_cols;
  if (nch == 0) return hipSuccess;
  // the squared exponential forms its distances on the matrix cores (gram.hip)
  if (h.kernel == KERNEL_SE && chunk_cols % 128 == 0)
    return launch_se_kmatvec_gram(A, rows, B, cols, d, h, v, partial, chunk_cols, st);
  dim3 grid((unsigned)((rows + KB - 1) / KB), (unsigned)nch);
  hipLaunchKernelGGL(kmatvec_partial_kernel, grid, dim3(256), 0, st, A, rows, B, cols, d, h, v, partial,
                     chunk_cols);
  return hipGetLastError();
}

}  // namespace gpr
