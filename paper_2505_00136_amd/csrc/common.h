// Shared device/host definitions of the gfx950 GP library (internal; not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#define GPR_DEV __device__ __forceinline__

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace gpr {

// ---------------------------------------------------------------- hyperparameters
// Kernels receive the hyperparameters by value; when `theta_log` is non-null they
// use exp(theta_log[0..2]) instead, so an optimisation loop can keep them on the device.
// `kernel` selects the covariance function (KERNEL_* below).
struct HyperArg {
  double ell, nu, s2;
  const double* theta_log;
  int kernel;
};

// Covariance functions: the squared exponential of Eq. 2 and the half-integer Matern
// kernels that Section 6 names as further kernel functions (s = r / l):
//   KERNEL_M12: nu exp(-s)
//   KERNEL_M32: nu (1 + sqrt(3) s) exp(-sqrt(3) s)
//   KERNEL_M52: nu (1 + sqrt(5) s + 5 s^2 / 3) exp(-sqrt(5) s)
enum { KERNEL_SE = 0, KERNEL_M12 = 1, KERNEL_M32 = 2, KERNEL_M52 = 3 };
constexpr double SQRT3 = 1.7320508075688772935, SQRT5 = 2.2360679774997896964;

// Evaluates the selected covariance function from squared distances; set up once per
// thread (the branch is uniform over a launch).
struct CovFn {
  int kernel;
  double nu, g, inv_ell;   // g = -1 / (2 l^2)
  GPR_DEV CovFn(int k, double ell, double nu_) : kernel(k), nu(nu_), g(-0.5 / (ell * ell)), inv_ell(1.0 / ell) {}
  GPR_DEV double operator()(double r2) const {
    if (kernel == KERNEL_SE) return nu * exp(g * r2);
    const double s = sqrt(r2) * inv_ell;
    if (kernel == KERNEL_M12) return nu * exp(-s);
    if (kernel == KERNEL_M32) {
      const double q = SQRT3 * s;
      return nu * (1.0 + q) * exp(-q);
    }
    const double q = SQRT5 * s;
    return nu * (1.0 + q + q * q * (1.0 / 3.0)) * exp(-q);
  }
};

// Matern value kf and its derivative with respect to log l from u = r^2 / (2 l^2)
// (s = sqrt(2u)): M12: nu s exp(-s); M32: 3 nu s^2 exp(-sqrt(3) s);
// M52: (5/3) nu s^2 (1 + sqrt(5) s) exp(-sqrt(5) s).
GPR_DEV void matern_and_dlogl(int kernel, double u, double nu, double& kf, double& dl) {
  const double s = sqrt(2.0 * u);
  if (kernel == KERNEL_M12) {
    const double e = nu * exp(-s);
    kf = e;
    dl = s * e;
  } else if (kernel == KERNEL_M32) {
    const double q = SQRT3 * s, e = nu * exp(-q);
    kf = (1.0 + q) * e;
    dl = q * q * e;
  } else {
    const double q = SQRT5 * s, e = nu * exp(-q);
    kf = (1.0 + q + q * q * (1.0 / 3.0)) * e;
    dl = q * q * (1.0 / 3.0) * (1.0 + q) * e;
  }
}

GPR_DEV void resolve_hyper(const HyperArg& h, double& ell, double& nu, double& s2) {
  if (h.theta_log) {
    ell = exp(h.theta_log[0]);
    nu = exp(h.theta_log[1]);
    s2 = exp(h.theta_log[2]);
  } else {
    ell = h.ell; nu = h.nu; s2 = h.s2;
  }
}

// ---------------------------------------------------------------- tiled matrix layout
// T x T tiles of b x b, lower triangle only.  Three regions, in this order:
//   D: T diagonal tiles, float64, row-major, tile k at k*b*b;
//   W: T diagonal-tile inverses L_kk^{-1} (float64, lower triangular), tile k at k*b*b;
//   O: T(T-1)/2 strictly-lower tiles in column-major packed order, element type `S`
//      (float64 for the FP64 path, float32 for the mixed paths); tile (i,j), i>j,
//      has index j(T-1) - j(j-1)/2 + (i-j-1), so the panel below a diagonal tile is contiguous.
// T = ceil(n / b).  When b does not divide n the matrix is padded to T b rows with an
// identity block: rows and columns n..Tb-1 are zero except for ones on the diagonal, so
// the factor is L of the n x n matrix bordered by that identity, its log-determinant is
// unchanged, and solves with zero-padded right-hand sides return zero padding.
// Tile pair (ti, tj), ti >= tj, of the row-major packed lower triangle y = ti (ti+1)/2 + tj.
GPR_DEV void pair_of(int64_t y, int64_t& ti, int64_t& tj) {
  ti = (int64_t)((sqrt(8.0 * (double)y + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= y) ++ti;
  while (ti * (ti + 1) / 2 > y) --ti;
  tj = y - ti * (ti + 1) / 2;
}

struct TileLayout {
  int64_t n, b, T;   // n: number of points (rows of Z), not necessarily T b
  int esize;  // bytes per element in region O (8 or 4)
  __host__ __device__ int64_t npad() const { return T * b; }
  // rows of Z behind tile row k (b, except in the last, partly padded tile)
  __host__ __device__ int64_t rows_of(int64_t k) const { return n - k * b < b ? n - k * b : b; }
  __host__ __device__ int64_t tile_elems() const { return b * b; }
  __host__ __device__ int64_t off_index(int64_t i, int64_t j) const {
    return j * (T - 1) - j * (j - 1) / 2 + (i - j - 1);
  }
  __host__ __device__ size_t d_bytes() const { return (size_t)T * b * b * 8; }
  __host__ __device__ size_t w_offset() const { return d_bytes(); }
  __host__ __device__ size_t o_offset() const { return 2 * d_bytes(); }
  __host__ __device__ size_t total_bytes() const {
    return 2 * d_bytes() + (size_t)(T * (T - 1) / 2) * b * b * esize;
  }
  __host__ __device__ double* diag(void* base, int64_t k) const {
    return (double*)base + k * b * b;
  }
  __host__ __device__ double* winv(void* base, int64_t k) const {
    return (double*)((char*)base + w_offset()) + k * b * b;
  }
  __host__ __device__ void* off(void* base, int64_t i, int64_t j) const {
    return (char*)base + o_offset() + (size_t)off_index(i, j) * b * b * esize;
  }
};

// ---------------------------------------------------------------- batched tile GEMM
// One job computes C[M x N] = alpha * sum_s op(A_s) op(B_s)^T + beta * Cin over its segments.
// Operand modes: element (r,k) of A is A[r*lda + k] (MODE_KC) or A[k*lda + r] (MODE_MC);
// element (c,k) of B is B[c*ldb + k] (MODE_KC) or B[k*ldb + c] (MODE_MC).
enum { MODE_KC = 0, MODE_MC = 1 };
// Triangular skips (the skipped products are exactly zero in memory):
//   A_LOWER: A(r,k) = 0 for k > r;  A_UPPER: A(r,k) = 0 for k < r;
//   B_LOWER: B(c,k) = 0 for k > c;  B_UPPER: B(c,k) = 0 for k < c.
enum { TRI_NONE = 0, A_LOWER = 1, A_UPPER = 2, B_LOWER = 4, B_UPPER = 8 };
// Job flags.
enum { JOB_LOWER_ONLY = 1,   // skip macro tiles that lie entirely above the diagonal
       JOB_C_F32 = 2,        // C and Cin are float32 (else float64)
       JOB_TRACE_ALPHA = 4 };  // gradient trace: this job also subtracts alpha alpha^T

struct GemmSeg {
  const void* A;
  const void* B;
  int64_t lda, ldb;
  int64_t pstrideA, pstrideB;   // element stride between the hi/mid/lo bfloat16 planes (split products)
  int32_t K;
  uint8_t modeA, modeB, tri, pad;
};

struct GemmJob {
  void* C;
  const void* Cin;
  int64_t ldc, ldcin;
  double alpha, beta;
  int32_t M, N;
  int32_t seg0, nseg;
  int32_t wg_begin;   // first workgroup of this job within its launch
  int32_t tiles_n;    // macro tiles along N
  int32_t flags;
  int32_t aux0, aux1;   // job-specific (the gradient reduction stores the tile indices here)
  int32_t pad;
};

// Arguments of the gradient reduction fused into the K^{-1} product.
struct TraceArgs {
  const double* u;       // r^2 / (2 l^2) of every lower tile pair (packed row-major, b x b each)
  const double* alpha;
  HyperArg h;
  int64_t b;
  double* partial;       // [workgroups][3]
};

constexpr int GEMM_BM = 128, GEMM_BN = 128, GEMM_THREADS = 256;   // macro tile, workgroup size

// Workgroup w is dispatched to XCD w % 8; remap so that every XCD gets a contiguous
// range of logical workgroups (neighbouring macro tiles share operands in that XCD's L2).
GPR_DEV int xcd_remap(int bid, int nblocks) {
  const int nx = 8;
  int xcd = bid % nx, local = bid / nx;
  int per = nblocks / nx, rem = nblocks % nx;
  int start = xcd * per + (xcd < rem ? xcd : rem);
  return start + local;
}

// Macro tile (m0, n0) of the job's t-th workgroup.  Tiles are visited in 8 x 8 blocks
// (row-major inside and between blocks) when the job's tile grid allows: consecutive
// workgroups land on one XCD (xcd_remap), and its ~64 resident workgroups then form a
// square patch that shares 8 A and 8 B row blocks through the XCD's L2 instead of a
// 4 x 16 strip sharing 4 and 16.
GPR_DEV void job_tile(const GemmJob& job, int t, int& m0, int& n0) {
  const int tn = job.tiles_n, tm = (job.M + GEMM_BM - 1) / GEMM_BM;
  if ((tn & 7) == 0 && (tm & 7) == 0) {
    const int sb = t >> 6, w = t & 63, sbn = tn >> 3;
    m0 = ((sb / sbn) * 8 + (w >> 3)) * GEMM_BM;
    n0 = ((sb % sbn) * 8 + (w & 7)) * GEMM_BN;
  } else {
    m0 = (t / tn) * GEMM_BM;
    n0 = (t % tn) * GEMM_BN;
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace gpr
