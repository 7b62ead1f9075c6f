// Host-side builder of a call's launch sequence (internal).
//
// A library call describes its work once through a Program: tile-GEMM jobs with
// their operand segments, interleaved with other kernel launches.  The call runs
// the description twice: a record pass that only collects the GEMM job tables
// (so their size is known and they can be copied to the device in one transfer),
// then an execute pass that launches everything in stream order, pointing each
// GEMM launch at its slice of the uploaded tables.
#pragma once
#include <functional>
#include <vector>
#include "common.h"
#include "kernels.h"

namespace gpr {

struct Program {
  bool exec = false;
  hipStream_t st = nullptr;
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  const GemmJob* djobs = nullptr;
  const GemmSeg* dsegs = nullptr;
  hipError_t err = hipSuccess;
  int64_t gemm_flops_wg = 0;   // workgroups launched (statistics)
  int job0 = 0, nwg = 0, f32 = 0;
  bool cur_valid = false;

  void reset_for_exec(const GemmJob* dj, const GemmSeg* ds) {
    exec = true;
    djobs = dj;
    dsegs = ds;
    jobs.clear();
    segs.clear();
  }
  size_t table_bytes() const { return jobs.size() * sizeof(GemmJob) + segs.size() * sizeof(GemmSeg) + 512; }

  void gemm_begin(int use_f32) {
    job0 = (int)jobs.size();
    nwg = 0;
    f32 = use_f32;
  }
  // Adds a job C[M x N] = alpha * sum(segments added next) + beta * Cin.
  void job(void* C, int64_t ldc, const void* Cin, int64_t ldcin, int64_t M, int64_t N, double alpha, double beta,
           int flags, int aux0 = 0, int aux1 = 0) {
    GemmJob j{};
    j.C = C;
    j.Cin = Cin;
    j.ldc = ldc;
    j.ldcin = ldcin;
    j.alpha = alpha;
    j.beta = beta;
    j.M = (int32_t)M;
    j.N = (int32_t)N;
    j.seg0 = (int32_t)segs.size();
    j.nseg = 0;
    j.wg_begin = nwg;
    j.tiles_n = (int32_t)ceil_div(N, GEMM_BN);
    j.flags = flags;
    j.aux0 = aux0;
    j.aux1 = aux1;
    cur_valid = M > 0 && N > 0;
    if (!cur_valid) return;
    const int64_t tiles = ceil_div(M, GEMM_BM) * (int64_t)j.tiles_n;
    jobs.push_back(j);
    nwg += (int)tiles;
  }
  void seg(const void* A, int64_t lda, int modeA, const void* B, int64_t ldb, int modeB, int64_t K, int tri = 0) {
    if (!cur_valid || K <= 0) return;
    GemmSeg s{};
    s.A = A;
    s.B = B;
    s.lda = lda;
    s.ldb = ldb;
    s.K = (int32_t)K;
    s.modeA = (uint8_t)modeA;
    s.modeB = (uint8_t)modeB;
    s.tri = (uint8_t)tri;
    segs.push_back(s);
    jobs.back().nseg++;
  }
  void gemm_end() {
    const int nj = (int)jobs.size() - job0;
    if (!exec || err != hipSuccess || nj == 0) return;
    gemm_flops_wg += nwg;
    err = launch_gemm(f32, djobs + job0, dsegs, nj, nwg, st);
  }
  // Launches produced by `fn` run only in the execute pass.
  void kernel(const std::function<hipError_t()>& fn) {
    if (!exec || err != hipSuccess) return;
    err = fn();
  }
};

}  // namespace gpr
