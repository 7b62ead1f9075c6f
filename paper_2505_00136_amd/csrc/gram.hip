// Squared-exponential kernel values (Eq. 2) with the squared distances from Gram products
// on the matrix cores -- fused kernel-vector products (posterior mean, Eq. 3, and the
// refinement residual), the tiled assembly and the gradient's scaled distances:
//   r_ij^2 = |a_i|^2 + |b_j|^2 - 2 a_i . b_j,
// the dot products of a 128 x 128 block of point pairs being one tile product with depth D
// (the tile-GEMM main loop of gemm_device.h, both operands k-contiguous: the rows of the
// row-major feature matrices).  The cancellation in this form costs an absolute error of a
// few ulp of |a|^2 + |b|^2 in r^2, i.e. a few times (|a|^2 + |b|^2) / (2 l^2) ulp of nu in
// the kernel value nu exp(-r^2 / (2 l^2)).  A block of pairs whose
// (max |a|^2 + max |b|^2) / (2 l^2) exceeds kGramRatioMax therefore forms its distances
// from explicit differences instead (features staged through LDS), which keeps the error
// of every kernel value at a few ulp of nu whatever the offset of the points from the
// origin; standardised features with l^2 near D (ratio about 1) take the Gram form.  The
// Matern forms, whose value depends on sqrt(r^2), keep the explicit differences of
// assemble.hip.  A pair of the same point (the training residual) gets r^2 = 0 exactly; a
// NaN feature makes every r^2 of its point NaN, as explicit differences do.
#include "common.h"
#include "gemm_device.h"
#include "kernels.h"

namespace gpr {

namespace {

constexpr double kGramRatioMax = 16.0;   // largest (max|a|^2 + max|b|^2) / (2 l^2) of the Gram form
constexpr int GR_WN = 4;                 // the tile-GEMM wave layout: 512 threads, 64 x 32 per wave
typedef Shape<GR_WN> GrShape;

// |P_r|^2 for rows r0 .. r0+127 of the row-major n x d matrix P (0 past `lim`), into nrm;
// four threads per row, fixed summation order.
GPR_DEV void row_norms(const double* __restrict__ P, int64_t lim, int64_t r0, int64_t d, double* nrm) {
  const int tid = threadIdx.x, r = tid >> 2, q = tid & 3;
  double s = 0.0;
  const int64_t row = r0 + r;
  if (row < lim) {
    const double* p = P + row * d;
    for (int64_t f = q; f < d; f += 4) s = fma(p[f], p[f], s);
  }
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  if (q == 0) nrm[r] = s;
}

// Largest of the 128 norms in nrm (wave 0 reduces, the result in *out).
GPR_DEV void max_norm(const double* nrm, double* out) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    double m = nrm[tid] > nrm[tid + 64] ? nrm[tid] : nrm[tid + 64];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double x = __shfl_xor(m, o);
      m = x > m ? x : m;
    }
    if (tid == 0) *out = m;
  }
}

constexpr int GR_FC = 32;   // features per LDS stage of the explicit differences

// acc[i][j][r] = sum_f (A_row - B_col)_f^2 for this lane's elements of the 128 x 128 block
// (the MFMA output layout of the Gram path), from explicit differences in feature order;
// rows past rlim and columns past clim read zero features.  Uses all of smem.
template <int NJ>
GPR_DEV void explicit_r2(const double* __restrict__ A, int64_t rlim, int64_t r0, const double* __restrict__ B,
                         int64_t clim, int64_t c0, int64_t d, char* smem, v4d (&acc)[4][NJ], int lane, int wm,
                         int wn) {
  double (*za)[GEMM_BM] = reinterpret_cast<double (*)[GEMM_BM]>(smem);
  double (*zb)[GEMM_BN] = za + GR_FC;
  const int tid = threadIdx.x, pr = tid >> 2, pf = (tid & 3) * 8;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = v4d{0, 0, 0, 0};
  for (int64_t f0 = 0; f0 < d; f0 += GR_FC) {
    __syncthreads();
    {
      const int64_t ga = r0 + pr, gb = c0 + pr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t f = f0 + pf + e;
        za[pf + e][pr] = (ga < rlim && f < d) ? A[ga * d + f] : 0.0;
        zb[pf + e][pr] = (gb < clim && f < d) ? B[gb * d + f] : 0.0;
      }
    }
    __syncthreads();
    const int fc = (int)((d - f0) < GR_FC ? (d - f0) : GR_FC);
    for (int f = 0; f < fc; ++f) {
      double b[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = zb[f][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double a = za[f][wm + i * 16 + MfmaOp<double>::row(lane, r)];
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const double df = a - b[j];
            acc[i][j][r] = fma(df, df, acc[i][j][r]);
          }
        }
    }
  }
  __syncthreads();   // the staging buffers are reused
}

}  // namespace

// partial[chunk][i] = sum over the chunk's points j of k(A_i, B_j) v_j (squared exponential).
// Grid (ceil(rows / 128), chunks); workgroup (x, y) takes rows 128 x .. and the points of
// chunk y in blocks of 128.  `same`: A and B are the same points (a pair (i, i) is at
// distance 0).
template <int SPEC>
__global__ __launch_bounds__(GrShape::THREADS, 2)
void se_kmatvec_gram_kernel(const double* __restrict__ A, int64_t rows, const double* __restrict__ B, int64_t cols,
                            int64_t d, HyperArg h, const double* __restrict__ v, double* __restrict__ partial,
                            int64_t chunk_cols, int same) {
  __shared__ __align__(16) char smem[Chunk<double>::SMEM];
  __shared__ double na[GEMM_BM], nb[GEMM_BN];
  __shared__ double red[GR_WN][GEMM_BM];
  __shared__ double maxna, maxnb;
  __shared__ GemmSeg seg;
  LdsBuf<double> As = reinterpret_cast<LdsBuf<double>>(smem);
  LdsBuf<double> Bs = As + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = GrShape::m0(wave), wn = GrShape::n0(wave);
  const int64_t r0 = (int64_t)blockIdx.x * GEMM_BM;
  const int64_t cbeg = (int64_t)blockIdx.y * chunk_cols;
  const int64_t cend = cbeg + chunk_cols < cols ? cbeg + chunk_cols : cols;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const double g = -0.5 / (ell * ell);
  if (tid == 0) seg = GemmSeg{A, B, d, d, 0, 0, (int32_t)d, MODE_KC, MODE_KC, 0, 0};
  if (tid < GR_WN * GEMM_BM) red[tid / GEMM_BM][tid % GEMM_BM] = 0.0;
  GemmJob job{};
  job.M = (int32_t)rows;
  job.N = (int32_t)cols;
  job.seg0 = 0;
  job.nseg = 1;
  row_norms(A, rows, r0, d, na);
  __syncthreads();
  max_norm(na, &maxna);
  for (int64_t c0 = cbeg; c0 < cend; c0 += GEMM_BN) {
    row_norms(B, cend, c0, d, nb);
    __syncthreads();
    max_norm(nb, &maxnb);
    __syncthreads();   // norms, their maxima and the segment visible; the previous block's LDS reads done
    v4d acc[4][GrShape::NJ];
    if ((maxna + maxnb) * (-g) <= kGramRatioMax) {
      // squared distances from the Gram products
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < GrShape::NJ; ++j) acc[i][j] = v4d{0, 0, 0, 0};
      gemm_mainloop<double, double, SPEC, GR_WN>(job, &seg, (int)r0, (int)c0, acc, As, Bs);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < GrShape::NJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double r2 = na[wm + i * 16 + MfmaOp<double>::row(lane, r)] + nb[wn + j * 16 + (lane & 15)] -
                              2.0 * acc[i][j][r];
            acc[i][j][r] = r2 < 0.0 ? 0.0 : r2;   // (a NaN stays NaN)
          }
    } else {
      explicit_r2<GrShape::NJ>(A, rows, r0, B, cend, c0, d, smem, acc, lane, wm, wn);
    }
    double vj[GrShape::NJ];
#pragma unroll
    for (int j = 0; j < GrShape::NJ; ++j) {
      const int64_t col = c0 + wn + j * 16 + (lane & 15);
      vj[j] = col < cend ? v[col] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = wm + i * 16 + MfmaOp<double>::row(lane, r);
        const int64_t row = r0 + lr;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < GrShape::NJ; ++j) {
          const int lc = wn + j * 16 + (lane & 15);
          const int64_t col = c0 + lc;
          double r2 = acc[i][j][r];
          if (same && row == col && r2 == r2) r2 = 0.0;   // a point with a NaN feature stays NaN
          if (row < rows && col < cend) s = fma(nu * exp(g * r2), vj[j], s);
        }
        // the 16 lanes holding this row (different columns), then one lane per row adds
        // the block's sum to its wave's slot
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        if ((lane & 15) == 0) red[wave % GR_WN][lr] += s;
      }
    __syncthreads();   // nb and the LDS operand buffers are rewritten by the next block
  }
  if (tid < GEMM_BM) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < GR_WN; ++q) s += red[q][tid];
    const int64_t r = r0 + tid;
    if (r < rows) partial[(int64_t)blockIdx.y * rows + r] = s;
  }
}

// The tiled covariance (OUT = 0, Eq. 2 with the identity padding of the tiled layout) or the
// gradient's u = r^2 / (2 l^2) tiles (OUT = 1) for the squared exponential, from the Gram
// products: workgroup x takes the 128 x 128 block x % nbt^2 of tile pair x / nbt^2 (row-
// major packed lower triangle of tile pairs).  Rows of a tile past its real points read
// zero features (their kernel values are replaced by the padding; their u, finite, gets
// zero weight in the gradient).  The Gram form's accuracy rule is the one of the products
// above: blocks with (max|a|^2 + max|b|^2) / (2 l^2) above kGramRatioMax take explicit
// differences.
template <int SPEC, int OUT>
__global__ __launch_bounds__(GrShape::THREADS, 4)   // two workgroups per CU: one's epilogue beside the other's products
void se_tiles_gram_kernel(const double* __restrict__ Z, int64_t d, HyperArg h, TileLayout L, void* K,
                          double* __restrict__ U) {
  __shared__ __align__(16) char smem[Chunk<double>::SMEM];
  __shared__ double na[GEMM_BM], nb[GEMM_BN];
  __shared__ double maxna, maxnb;
  __shared__ GemmSeg seg;
  LdsBuf<double> As = reinterpret_cast<LdsBuf<double>>(smem);
  LdsBuf<double> Bs = As + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = GrShape::m0(wave), wn = GrShape::n0(wave);
  const int64_t b = L.b, nbt = (b + GEMM_BM - 1) / GEMM_BM;
  const int64_t y = (int64_t)blockIdx.x / (nbt * nbt), blk = (int64_t)blockIdx.x % (nbt * nbt);
  int64_t ti, tj;
  pair_of(y, ti, tj);
  const int64_t r0 = (blk / nbt) * GEMM_BM, c0 = (blk % nbt) * GEMM_BN;   // within the tile
  const int64_t ri = L.rows_of(ti), rj = L.rows_of(tj);                   // real rows of the two tiles
  const double* A = Z + ti * b * d;
  const double* B = Z + tj * b * d;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const double g = -0.5 / (ell * ell);
  if (tid == 0) seg = GemmSeg{A, B, d, d, 0, 0, (int32_t)d, MODE_KC, MODE_KC, 0, 0};
  GemmJob job{};
  job.M = (int32_t)ri;
  job.N = (int32_t)rj;
  job.seg0 = 0;
  job.nseg = 1;
  row_norms(A, ri, r0, d, na);
  row_norms(B, rj, c0, d, nb);
  __syncthreads();
  max_norm(na, &maxna);
  __syncthreads();
  max_norm(nb, &maxnb);
  __syncthreads();
  v4d acc[4][GrShape::NJ];
  if ((maxna + maxnb) * (-g) <= kGramRatioMax) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j) acc[i][j] = v4d{0, 0, 0, 0};
    gemm_mainloop<double, double, SPEC, GR_WN>(job, &seg, (int)r0, (int)c0, acc, As, Bs);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double r2 = na[wm + i * 16 + MfmaOp<double>::row(lane, r)] + nb[wn + j * 16 + (lane & 15)] -
                            2.0 * acc[i][j][r];
          acc[i][j][r] = r2 < 0.0 ? 0.0 : r2;   // (a NaN stays NaN)
        }
  } else {
    explicit_r2<GrShape::NJ>(A, ri, r0, B, rj, c0, d, smem, acc, lane, wm, wn);
  }
  const bool diag = ti == tj;
  double* Dt = (OUT == 0 && diag) ? L.diag(K, ti) : nullptr;
  void* Ot = (OUT == 0 && !diag) ? L.off(K, ti, tj) : nullptr;
  double* Ut = OUT == 1 ? U + y * b * b : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wm + i * 16 + MfmaOp<double>::row(lane, r);
      if (row >= b) continue;
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j) {
        const int64_t col = c0 + wn + j * 16 + (lane & 15);
        if (col >= b) continue;
        double r2 = acc[i][j][r];
        if (diag && row == col && r2 == r2) r2 = 0.0;   // a point with a NaN feature stays NaN
        if (OUT == 1) {
          Ut[row * b + col] = -g * r2;
        } else {
          double v = nu * exp(g * r2);
          if (row >= ri || col >= rj) v = 0.0;   // padding: identity block, zero border
          if (diag) {
            if (row == col) v = row < ri ? v + s2 : 1.0;
            Dt[row * b + col] = v;
          } else if (L.esize == 8) {
            ((double*)Ot)[row * b + col] = v;
          } else {
            ((float*)Ot)[row * b + col] = (float)v;
          }
        }
      }
    }
}

hipError_t launch_se_tiles_gram(const double* Z, int64_t d, HyperArg h, const TileLayout& L, void* K, double* U,
                                hipStream_t st) {
  if (L.T == 0) return hipSuccess;
  if ((K == nullptr) == (U == nullptr) || d > 0x7fffffff || L.b > 0x7fffff00) return hipErrorInvalidValue;
  const int64_t nbt = (L.b + GEMM_BM - 1) / GEMM_BM;
  const int64_t blocks = nbt * nbt * (L.T * (L.T + 1) / 2);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  // the straight-line main loop: whole 128-point blocks in every tile (no padding), whole
  // 16-deep chunks, 16-byte aligned rows
  const bool full = L.b % GEMM_BM == 0 && L.n == L.npad() && d % Chunk<double>::BK == 0 && ((uintptr_t)Z & 15) == 0;
  const dim3 grid((unsigned)blocks), blk(GrShape::THREADS);
  if (U) {
    if (full) hipLaunchKernelGGL((se_tiles_gram_kernel<SPEC_KK, 1>), grid, blk, 0, st, Z, d, h, L, K, U);
    else hipLaunchKernelGGL((se_tiles_gram_kernel<SPEC_GUARDED, 1>), grid, blk, 0, st, Z, d, h, L, K, U);
  } else {
    if (full) hipLaunchKernelGGL((se_tiles_gram_kernel<SPEC_KK, 0>), grid, blk, 0, st, Z, d, h, L, K, U);
    else hipLaunchKernelGGL((se_tiles_gram_kernel<SPEC_GUARDED, 0>), grid, blk, 0, st, Z, d, h, L, K, U);
  }
  return hipGetLastError();
}

hipError_t launch_se_kmatvec_gram(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                  HyperArg h, const double* v, double* partial, int64_t chunk_cols, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  if (rows > 0x7fffff00 || cols > 0x7fffff00 || d > 0x7fffffff || chunk_cols % GEMM_BN != 0)
    return hipErrorInvalidValue;
  const int64_t nch = (cols + chunk_cols - 1) / chunk_cols;
  dim3 grid((unsigned)((rows + GEMM_BM - 1) / GEMM_BM), (unsigned)nch);
  const int same = (A == B && rows == cols) ? 1 : 0;
  // the straight-line main loop needs whole 128-point blocks, whole 16-deep chunks and
  // 16-byte aligned rows; anything else takes the guarded loop
  const bool full = rows % GEMM_BM == 0 && cols % GEMM_BN == 0 && d % Chunk<double>::BK == 0 &&
                    ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
  if (full)
    hipLaunchKernelGGL(se_kmatvec_gram_kernel<SPEC_KK>, grid, dim3(GrShape::THREADS), 0, st, A, rows, B, cols, d, h,
                       v, partial, chunk_cols, same);
  else
    hipLaunchKernelGGL(se_kmatvec_gram_kernel<SPEC_GUARDED>, grid, dim3(GrShape::THREADS), 0, st, A, rows, B, cols, d,
                       h, v, partial, chunk_cols, same);
  return hipGetLastError();
}

// The refinement's K v with the symmetry of K (A = B = Z): one 128 x 128 block of the
// lower triangle per workgroup (block pair y = bi (bi+1)/2 + bj, bj <= bi), two workgroups
// per CU.  Its row sums sum_j k_ij v_j go to rowpart[bj][i] for its rows i and, below the
// diagonal, its column sums sum_i k_ij v_i to colpart[bi][j] for its columns j; each entry
// is written by one workgroup, and row i of K v is the sum of rowpart[bj][i] over
// bj <= i / 128 and colpart[x][i] over x > i / 128 (launch_residual_finish_sym).
template <int SPEC>
__global__ __launch_bounds__(GrShape::THREADS, 4)
void se_kmatvec_sym_kernel(const double* __restrict__ Z, int64_t n, int64_t d, HyperArg h,
                           const double* __restrict__ v, double* __restrict__ rowpart, double* __restrict__ colpart) {
  __shared__ __align__(16) char smem[Chunk<double>::SMEM];
  __shared__ double na[GEMM_BM], nb[GEMM_BN], va[GEMM_BM], vb[GEMM_BN];
  __shared__ double red[GR_WN][GEMM_BM], cred[2][GEMM_BN];
  __shared__ double maxna, maxnb;
  __shared__ GemmSeg seg;
  LdsBuf<double> As = reinterpret_cast<LdsBuf<double>>(smem);
  LdsBuf<double> Bs = As + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = GrShape::m0(wave), wn = GrShape::n0(wave);
  int64_t bi, bj;
  pair_of((int64_t)blockIdx.x, bi, bj);
  const int64_t r0 = bi * GEMM_BM, c0 = bj * GEMM_BN;
  const bool diag = bi == bj;
  double ell, nu, s2;
  resolve_hyper(h, ell, nu, s2);
  const double g = -0.5 / (ell * ell);
  if (tid == 0) seg = GemmSeg{Z, Z, d, d, 0, 0, (int32_t)d, MODE_KC, MODE_KC, 0, 0};
  if (tid < GEMM_BM) va[tid] = r0 + tid < n ? v[r0 + tid] : 0.0;
  if (tid >= GEMM_BM && tid < GEMM_BM + GEMM_BN) {
    const int t = tid - GEMM_BM;
    vb[t] = c0 + t < n ? v[c0 + t] : 0.0;
  }
  GemmJob job{};
  job.M = (int32_t)n;
  job.N = (int32_t)n;
  job.seg0 = 0;
  job.nseg = 1;
  row_norms(Z, n, r0, d, na);
  row_norms(Z, n, c0, d, nb);
  __syncthreads();
  max_norm(na, &maxna);
  __syncthreads();
  max_norm(nb, &maxnb);
  __syncthreads();
  v4d acc[4][GrShape::NJ];
  if ((maxna + maxnb) * (-g) <= kGramRatioMax) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j) acc[i][j] = v4d{0, 0, 0, 0};
    gemm_mainloop<double, double, SPEC, GR_WN>(job, &seg, (int)r0, (int)c0, acc, As, Bs);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double r2 = na[wm + i * 16 + MfmaOp<double>::row(lane, r)] + nb[wn + j * 16 + (lane & 15)] -
                            2.0 * acc[i][j][r];
          acc[i][j][r] = r2 < 0.0 ? 0.0 : r2;   // (a NaN stays NaN)
        }
  } else {
    explicit_r2<GrShape::NJ>(Z, n, r0, Z, n, c0, d, smem, acc, lane, wm, wn);
  }
  double cs[GrShape::NJ];
#pragma unroll
  for (int j = 0; j < GrShape::NJ; ++j) cs[j] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = wm + i * 16 + MfmaOp<double>::row(lane, r);
      const int64_t row = r0 + lr;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < GrShape::NJ; ++j) {
        const int lc = wn + j * 16 + (lane & 15);
        const int64_t col = c0 + lc;
        double r2 = acc[i][j][r];
        if (diag && row == col && r2 == r2) r2 = 0.0;   // a point with a NaN feature stays NaN
        if (row < n && col < n) {
          const double kv = nu * exp(g * r2);
          s = fma(kv, vb[lc], s);
          if (!diag) cs[j] = fma(kv, va[lr], cs[j]);
        }
      }
      // the 16 lanes holding this row (different columns); one lane per row writes its
      // wave's sum (the waves of one column range hold different rows)
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
      if ((lane & 15) == 0) red[wave % GR_WN][lr] = s;
    }
  if (!diag) {
    // the four lanes holding each column (rows 16 apart), then the two waves of each
    // column range (rows 0-63 and 64-127)
#pragma unroll
    for (int j = 0; j < GrShape::NJ; ++j) {
      cs[j] += __shfl_xor(cs[j], 16);
      cs[j] += __shfl_xor(cs[j], 32);
      if (lane < 16) cred[wave / GR_WN][wn + j * 16 + lane] = cs[j];
    }
  }
  __syncthreads();
  if (tid < GEMM_BM && r0 + tid < n) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < GR_WN; ++q) t += red[q][tid];
    rowpart[bj * n + r0 + tid] = t;
  }
  if (!diag && tid >= GEMM_BM && tid < GEMM_BM + GEMM_BN && c0 + (tid - GEMM_BM) < n) {
    const int t = tid - GEMM_BM;
    colpart[bi * n + c0 + t] = cred[0][t] + cred[1][t];
  }
}

hipError_t launch_se_kmatvec_gram_sym(const double* Z, int64_t n, int64_t d, HyperArg h, const double* v,
                                      double* rowpart, double* colpart, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n > 0x7fffff00 || d > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t nbk = (n + GEMM_BM - 1) / GEMM_BM;
  const int64_t blocks = nbk * (nbk + 1) / 2;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const bool full = n % GEMM_BM == 0 && d % Chunk<double>::BK == 0 && ((uintptr_t)Z & 15) == 0;
  if (full)
    hipLaunchKernelGGL((se_kmatvec_sym_kernel<SPEC_KK>), dim3((unsigned)blocks), dim3(GrShape::THREADS), 0, st, Z, n,
                       d, h, v, rowpart, colpart);
  else
    hipLaunchKernelGGL((se_kmatvec_sym_kernel<SPEC_GUARDED>), dim3((unsigned)blocks), dim3(GrShape::THREADS), 0, st,
                       Z, n, d, h, v, rowpart, colpart);
  return hipGetLastError();
}

}  // namespace gpr
