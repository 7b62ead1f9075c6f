// Factorisation and inversion of one diagonal block (up to 64 x 64) by one workgroup
// (device code, internal; used by potrf_block.hip and the task-graph executor of dag.hip).
//
// The diagonal tile of each step of the tiled factorisation (the POTRF task of
// Fig. 1) is factored by a blocked right-looking loop over 64-wide blocks (the
// orchestration issues the block steps in stream order); this kernel handles the
// diagonal block of each block step.  The block and its inverse live in registers:
// TPR threads per row (4 in the kernel of its own, 8 in the task-graph executor), thread
// t owns row t/TPR and every TPR-th column starting at t%TPR, of both A (becoming L) and
// W = L^{-1}.  Column j is eliminated with unscaled operands:
// with a = column j of A and w = row j of W as they stand after step j-1,
// l_ij l_kj = a_ij a_kj / a_jj and l_ij W_jc = a_ij w_c / a_jj, so each row i > j updates
//   A_ik -= c a_kj  and  W_ic -= c w_c,   c = a_ij (1/L_jj)^2,
// the right-looking Cholesky fused with forward elimination of L W = I.  Column k of A
// and row i of W keep their unscaled values in registers until the final store applies
// 1/L_kk and 1/L_ii.  One barrier per column: the threads that update column j+1 during
// step j publish it (and the row of W that step j finishes, and the next pivot) into the
// other half of double-buffered LDS exchange vectors, which are zero outside their ranges
// (a_kj for k > j, w_c for c <= j), so the updates run unmasked over all of a thread's
// columns (the entries they leave wrong, k > i, are never stored) and no register is
// indexed at run time.
#pragma once
#include "common.h"

namespace gpr {

// Block edge PB, PB * TPR working threads (TPR threads per row); thread t owns row t / TPR
// and columns t % TPR + TPR q.  The elimination applies the same operations to every
// element whatever TPR is, so the results do not depend on it.  Threads with
// tid >= PB * TPR (in a larger workgroup) only take part in the barriers.
// smem: potrf_block_smem<PB>() bytes of LDS.
template <int PB>
constexpr int potrf_block_smem() { return (2 * 2 * PB + 2 * PB) * (int)sizeof(double); }

template <int PB, int TPR>
GPR_DEV void potrf_block_work(double* __restrict__ A, int64_t lda, double* __restrict__ W, int64_t ldw, int jb,
                              int64_t col_base, unsigned long long* info, int tid, char* smem) {
  constexpr int PQ = PB / TPR;
  static_assert(PQ % 2 == 0, "columns per thread come in pairs");
  // exchange vectors of step j in buffer j % 2, element k stored at [k % TPR][k / TPR] so
  // that each thread's operands are contiguous: exl = column j of A (zero for k <= j),
  // exw = row j of W (zero for c > j)
  double (*exl)[TPR][PQ] = reinterpret_cast<double (*)[TPR][PQ]>(smem);
  double (*exw)[TPR][PQ] = exl + 2;
  double* piv = reinterpret_cast<double*>(exw + 2);
  double* ipiv = piv + PB;
  const bool active = tid < PB * TPR;
  const int i = active ? tid / TPR : PB, cq = tid % TPR;
  double ra[PQ], rw[PQ];
#pragma unroll
  for (int q = 0; q < PQ; ++q) {
    const int k = cq + TPR * q;
    ra[q] = (i < jb && k <= i) ? A[(int64_t)i * lda + k] : 0.0;
    rw[q] = (i < jb && k == i) ? 1.0 : 0.0;
  }
  // step 0's operands: column 0 of A below the diagonal, row 0 of W, the first pivot
  if (active && cq == 0) exl[0][i % TPR][i / TPR] = (i > 0 && i < jb) ? ra[0] : 0.0;
  if (active && i == 0) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) exw[0][cq][q] = rw[q];
    if (cq == 0) {
      const double d = ra[0];
      if (!(d > 0.0)) atomicMin(info, (unsigned long long)(col_base + 1));
      const double p = sqrt(d);
      piv[0] = p;
      ipiv[0] = 1.0 / p;
    }
  }
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    const int cur = j & 1, nxt = cur ^ 1, j1 = j + 1;
    const bool owner = active && cq == (j1 % TPR);   // this thread holds column j+1 of its row
    if (active && i > j && i < jb) {
      const double inv = ipiv[j];
      const double c = exl[cur][i % TPR][i / TPR] * (inv * inv);
      double el[PQ], ew[PQ];
#pragma unroll
      for (int q = 0; q < PQ; q += 2) {
        const double2 vl = *reinterpret_cast<const double2*>(&exl[cur][cq][q]);
        const double2 vw = *reinterpret_cast<const double2*>(&exw[cur][cq][q]);
        el[q] = vl.x;
        el[q + 1] = vl.y;
        ew[q] = vw.x;
        ew[q + 1] = vw.y;
      }
      double nv = 0.0;
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        ra[q] = fma(-c, el[q], ra[q]);
        rw[q] = fma(-c, ew[q], rw[q]);
        nv = (cq + TPR * q == j1) ? ra[q] : nv;
      }
      if (owner) {
        exl[nxt][i % TPR][i / TPR] = i > j1 ? nv : 0.0;
        if (i == j1) {
          if (!(nv > 0.0)) atomicMin(info, (unsigned long long)(col_base + j1 + 1));
          const double p = sqrt(nv);
          piv[j1] = p;
          ipiv[j1] = 1.0 / p;
        }
      }
      if (i == j1) {                                        // row j+1 of W is final (unscaled)
#pragma unroll
        for (int q = 0; q < PQ; ++q) exw[nxt][cq][q] = rw[q];
      }
    } else if (owner) {
      exl[nxt][i % TPR][i / TPR] = 0.0;
    }
    __syncthreads();
  }
  // column k of A and row i of W kept their unscaled values in the registers
#pragma unroll
  for (int q = 0; q < PQ; ++q) {
    const int k = cq + TPR * q;
    if (i < jb && k < jb) {
      A[(int64_t)i * lda + k] = k < i ? ra[q] * ipiv[k] : (k == i ? piv[k] : 0.0);
      W[(int64_t)i * ldw + k] = k <= i ? rw[q] * ipiv[i] : 0.0;
    }
  }
}

}  // namespace gpr
