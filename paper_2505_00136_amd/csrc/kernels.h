// Host-side launchers of the gfx950 kernels (internal; not part of the C-ABI).
#pragma once
#include <vector>

#include "common.h"
#include "dag.h"

namespace gpr {

// gemm.hip / gemm_bf16.hip
// GENERIC/UPDATE: operands and products in the launch precision; WIDEN: float32 operands,
// float64 products; BF16X3/X6: split-bfloat16 products of bfloat16 planes.
enum { GEMM_KIND_GENERIC = 0, GEMM_KIND_UPDATE = 1, GEMM_KIND_BF16X3 = 2, GEMM_KIND_BF16X6 = 3, GEMM_KIND_WIDEN = 4,
       GEMM_KIND_TRTRI = 5,    // triangular-inverse steps of the gradient (own kernel symbol)
       GEMM_KIND_TRACE = 6,    // K^{-1} products fused with the gradient reduction (launch_gemm_trace)
       // split-bfloat16 update on 256 x 256 macro tiles from planes in the tiled layout
       // (gemm_bf16.hip; tiles whose edge is a multiple of 256)
       GEMM_KIND_BF16X3_T256 = 7, GEMM_KIND_BF16X6_T256 = 8,
       // the gradient's inversion steps and fused trace products from split-bfloat16 planes
       // on 256 x 256 macro tiles (own kernel symbols)
       GEMM_KIND_BF16X3_TRTRI_T256 = 9, GEMM_KIND_BF16X6_TRTRI_T256 = 10,
       GEMM_KIND_BF16X3_TRACE_T256 = 11, GEMM_KIND_BF16X6_TRACE_T256 = 12,
       // the variance's forward substitution (own kernel symbols, not timed)
       GEMM_KIND_BF16X3_SOLVE_T256 = 13, GEMM_KIND_BF16X6_SOLVE_T256 = 14 };
inline bool gemm_kind_bf16(int kind) {
  return kind == GEMM_KIND_BF16X3 || kind == GEMM_KIND_BF16X6 || (kind >= GEMM_KIND_BF16X3_T256 && kind <= 14);
}
inline int gemm_kind_nprod(int kind) {
  return (kind == GEMM_KIND_BF16X6 || kind == GEMM_KIND_BF16X6_T256 || kind == GEMM_KIND_BF16X6_TRTRI_T256 ||
          kind == GEMM_KIND_BF16X6_TRACE_T256 || kind == GEMM_KIND_BF16X6_SOLVE_T256)
             ? 6
             : 3;
}
inline bool gemm_kind_solve(int kind) {
  return kind == GEMM_KIND_BF16X3_SOLVE_T256 || kind == GEMM_KIND_BF16X6_SOLVE_T256;
}
inline bool gemm_kind_trtri(int kind) {
  return kind == GEMM_KIND_TRTRI || kind == GEMM_KIND_BF16X3_TRTRI_T256 || kind == GEMM_KIND_BF16X6_TRTRI_T256;
}
inline bool gemm_kind_trace(int kind) {
  return kind == GEMM_KIND_TRACE || kind == GEMM_KIND_BF16X3_TRACE_T256 || kind == GEMM_KIND_BF16X6_TRACE_T256;
}
// macro tile edge of a launch of this kind (the workgroup count of each job follows from it)
inline int gemm_kind_macro(int kind) { return kind >= GEMM_KIND_BF16X3_T256 && kind <= 14 ? 256 : GEMM_BM; }
// spec: main-loop specialisation from gemm_launch_spec (host tables of the launch)
hipError_t launch_gemm(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int kind, int spec,
                       hipStream_t st);
hipError_t launch_gemm_trace(int prec_f32, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, int spec,
                             const TraceArgs& ta, hipStream_t st);
// Straight-line main loop of one operand-mode pair (0: KC/KC, 1: KC/MC, 3: MC/MC) when every
// job covers whole 128 x 128 macro tiles and every segment has K a multiple of the chunk
// depth bk of the main loop, 16-byte aligned rows and that pair;
// -1 (guarded loop) otherwise.  esize: bytes per stored operand element.
int gemm_launch_spec(const GemmJob* jobs, int njobs, const GemmSeg* segs, int esize, int bk);

// gemm_bf16.hip: trailing update from split-bfloat16 planes (nprod 3 or 6); KC operands only
hipError_t launch_gemm_bf16(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, hipStream_t st);
// hi/mid/lo bfloat16 parts (round to nearest even) of float32 x; lo may be null
hipError_t launch_split_bf16x3(const float* x, int64_t count, void* hi, void* mid, void* lo, hipStream_t st);
// the same for b x b row-major tiles (count a multiple of b^2, b % 256 == 0), the parts
// written in the tiled layout of the 256 x 256 update kernel
hipError_t launch_split_bf16x3_tiled(const float* x, int64_t count, int64_t b, void* hi, void* mid, void* lo,
                                     hipStream_t st);
// the update on 256 x 256 macro tiles (jobs of whole macro tiles, tiled-layout planes)
hipError_t launch_gemm_bf16_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                 hipStream_t st);

// the gradient's inversion steps and fused trace products on 256 x 256 macro tiles
hipError_t launch_gemm_bf16_trtri_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       hipStream_t st);
hipError_t launch_gemm_bf16_trace_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       const TraceArgs& ta, hipStream_t st);
// the variance's forward substitution on 256 x 256 macro tiles
hipError_t launch_gemm_bf16_solve_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       hipStream_t st);
// planes (2 or 3) of nblocks rows x kd operands (rows % 256 == 0, kd % 16 == 0) read from
// float32 row-major blocks at the given (16-byte aligned) addresses with leading dimension
// ld, as stored or transposed (trans: operand element (r, c) is source element (c, r)), in
// the tiled layout; block t at out + t rows kd of each plane, plane stride pstride
// elements (a multiple of 8)
hipError_t launch_split_bf16_tiles(const float* const* blocks, int64_t nblocks, int64_t rows, int64_t kd, int64_t ld,
                                   bool trans, void* out, int64_t pstride, int np, hipStream_t st);

// potrf_block.hip: Cholesky + inverse of one jb x jb (jb <= 64) diagonal block by one workgroup
hipError_t launch_potrf_block(double* A, int64_t lda, double* W, int64_t ldw, int jb, int64_t col_base,
                              unsigned long long* info, hipStream_t st);

// potrf.hip
hipError_t launch_set_identity(double* W, int64_t b, hipStream_t st);
hipError_t launch_zero_upper(double* A, int64_t b, hipStream_t st);
hipError_t launch_convert_f64_f32(const double* src, float* dst, int64_t count, hipStream_t st);
// device copy with a kernel on `st` (16-byte vectors when aligned)
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count, hipStream_t st);
// dst tile t = transpose of src tile t, t < count, b x b row-major tiles of esize (4 or 8) bytes
hipError_t launch_transpose_tiles(const void* src, void* dst, int64_t b, int64_t count, int esize, hipStream_t st);
// dst tile j = transpose of tile (row, j) of region O (T x T tiles at obase), j < row
hipError_t launch_transpose_block_row(const void* obase, int64_t T, int64_t row, void* dst, int64_t b, int esize,
                                      hipStream_t st);
// zero `bytes` bytes at p (4-byte aligned pointer and size) with a kernel
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// assemble.hip
// Lower tiles of K (Eq. 2) into the tiled layout: region D (float64) and region O (esize 8 or 4).
hipError_t launch_assemble_tiles(const double* Z, int64_t d, HyperArg h, const TileLayout& L, void* K,
                                 hipStream_t st);
// Dense covariance block out[r*ld + c] = k(A_r, B_c) (+ s2 where r == c when add_diag), float64 or float32.
// u = r^2 / (2 l^2) of every lower tile pair (T (T+1)/2 float64 b x b tiles, packed row-major);
// Z has n rows, (T-1) b < n <= T b, padded rows read as zero features
hipError_t launch_halfdist_tiles(const double* Z, int64_t n, int64_t d, HyperArg h, int64_t b, int64_t T, double* U,
                                 hipStream_t st);
hipError_t launch_assemble_dense(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                 HyperArg h, int add_diag, void* out, int64_t ld, int out_f32,
                                 hipStream_t st);
// partial[chunk][i] = sum over points j of chunk: k(A_i, B_j) v_j  (float64)
hipError_t launch_kmatvec_partial(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                  HyperArg h, const double* v, double* partial, int64_t chunk_cols,
                                  hipStream_t st);
// the same for the squared exponential, the distances from Gram products on the matrix
// cores (gram.hip); chunk_cols a multiple of 128
hipError_t launch_se_kmatvec_gram(const double* A, int64_t rows, const double* B, int64_t cols, int64_t d,
                                  HyperArg h, const double* v, double* partial, int64_t chunk_cols, hipStream_t st);
// The tiled covariance (K != null; layout L, as launch_assemble_tiles) or the gradient's
// u = r^2 / (2 l^2) tiles of every lower tile pair (U != null; L.esize ignored), squared
// exponential, distances from Gram products on the matrix cores (gram.hip)
hipError_t launch_se_tiles_gram(const double* Z, int64_t d, HyperArg h, const TileLayout& L, void* K, double* U,
                                hipStream_t st);
// The refinement's K v for the squared exponential with the symmetry of K: Z (n x d) against
// itself, one 128 x 128 block of the lower triangle per workgroup; rowpart[ceil(n / 128)][n]
// (row sums of each block column) and colpart[ceil(n / 128)][n] (column sums of the blocks
// below the diagonal), combined by launch_residual_finish_sym
hipError_t launch_se_kmatvec_gram_sym(const double* Z, int64_t n, int64_t d, HyperArg h, const double* v,
                                      double* rowpart, double* colpart, hipStream_t st);

// blas2.hip
// y[r] = beta*yin[r] + alpha * sum_c A[r*lda + c] x[c]   for r < rows (A float64 or float32)
hipError_t launch_gemv_n(const void* A, int a_f32, int64_t lda, int64_t rows, int64_t cols,
                         const double* x, double alpha, const double* yin, double beta, double* y,
                         hipStream_t st);
// partial[ch][c] = sum_{r in chunk ch} A[r*lda + c] x[r]
hipError_t launch_gemv_t_partial(const void* A, int a_f32, int64_t lda, int64_t rows, int64_t cols,
                                 const double* x, double* partial, int64_t rows_per_chunk,
                                 hipStream_t st);
// y[c] = beta*yin[c] + alpha * sum_ch partial[ch][c]    (fixed order)
hipError_t launch_reduce_partials(const double* partial, int64_t nch, int64_t cols, double alpha,
                                  const double* yin, double beta, double* y, hipStream_t st);
// colsq partial: partial[ch][c] = sum_{r in chunk} V[r*ld + c]^2
hipError_t launch_colsq_partial(const void* V, int v_f32, int64_t ld, int64_t rows, int64_t cols,
                                double* partial, int64_t rows_per_chunk, hipStream_t st);
// out[c] = nu (+ s2 if add_noise) - sum_ch partial[ch][c]
hipError_t launch_var_finish(const double* partial, int64_t nch, int64_t cols, HyperArg h, int add_noise,
                             double* out, hipStream_t st);
// nlml = 1/2 y.alpha + sum_i log L_ii + n/2 log 2 pi over i < n (L_ii read from the diagonal tiles)
hipError_t launch_nlml(const double* Ddiag, int64_t b, int64_t n, const double* y, const double* alpha,
                       double* nlml, hipStream_t st);
// r = y - (Kf alpha + s2 alpha) from partial K_f alpha sums
hipError_t launch_residual_finish(const double* partial, int64_t nch, int64_t n, HyperArg h,
                                  const double* y, const double* alpha, double* r, hipStream_t st);
// r = y - (K alpha + sigma^2 alpha) from the symmetric products (launch_se_kmatvec_gram_sym):
// row i adds rowpart[bj][i] for bj <= i / 128, then colpart[x][i] for x > i / 128
hipError_t launch_residual_finish_sym(const double* rowpart, const double* colpart, int64_t n, HyperArg h,
                                      const double* y, const double* alpha, double* r, hipStream_t st);
// grad[k] = trainable[k] ? 1/2 * (s_l, s_nu, s2 * s_s)[k] : 0, from per-workgroup partials;
// npadded padded rows each added exactly nu to s_nu and 1 to s_s, which are taken off
hipError_t launch_grad_finish(const double* partial, int64_t nwg, HyperArg h, int64_t npadded, int t0, int t1,
                              int t2, double* grad, hipStream_t st);
// One Adam step on theta_log[3] with state m[3], v[3], t (device), masked by trainable.
hipError_t launch_adam3(double* theta, double* state, const double* grad, double lr, double b1, double b2,
                        double eps, int t0, int t1, int t2, hipStream_t st);
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st);

// dag.hip: the persistent executor of a task graph (dag.h) on `st`, with `slots`
// workgroups (dag_slots: as many as fit on the device at once) and its run state at
// `state` (dag_state_ints(ntasks) int32); when no task finishes for limit_s seconds the run
// gives up and DAG_ABORT_INFO is left in info[0].
hipError_t dag_slots(int* slots);
hipError_t launch_dag(const DagTask* tasks, int ntasks, const int32_t* succ, const DagOp* ops, const GemmJob* jobs,
                      const GemmSeg* segs, int32_t* state, unsigned long long* info, double limit_s, int slots,
                      hipStream_t st);

// scratch.hip: file-scope device array of kScratchDoubles float64 (the partial sums of the
// allocation-free prediction); scratch_setup() looks up its address on the current device
// (once per device, then cached) and returns it in *out (out may be null).
constexpr int64_t kScratchDoubles = (int64_t)1 << 21;   // 16 MiB per device
hipError_t scratch_setup(double** out);

// warmstart.hip
int64_t stats_sort_len(int64_t nsub);
hipError_t launch_summary_stats(const double* Zraw, const double* Zstd, const double* yraw, int64_t n, int64_t d,
                                const int64_t* sub, int64_t nsub, double* work, double* out64, float* out32,
                                hipStream_t st);
int mlp_nparams();
size_t mlp_act_floats(int B);
hipError_t launch_mlp(float* params, float* m, float* v, float* grad, const float* X, const float* Y, float* out,
                      float* loss, float* act, int B, int mode, float lr, float b1, float b2, float eps, int t,
                      hipStream_t st);

}  // namespace gpr
