// Device code of the batched tile GEMM (internal), shared by the launch-per-step kernels
// of gemm.hip and the device-side task-graph executor of dag.hip.
//
// A workgroup computes one 128x128 macro tile of one job with 2 x WN wave64s, each
// owning a 64 x (128/WN) block held as 4 x (8/WN) accumulators of the 16x16x4 MFMA.
// Operands are staged through double-buffered LDS in 16-deep K chunks (one barrier per
// chunk), the next chunk's global loads being in flight while the current one is
// multiplied.  LDS holds both operands k-major ([k][m]), so an MFMA fragment read by 16
// consecutive lanes touches 16 consecutive words.
#pragma once
#include "common.h"

namespace gpr {

// Workgroup shape: 2 x WN wave64s over the 128 x 128 macro tile.
template <int WN>
struct Shape {
  static constexpr int THREADS = 128 * WN;
  static constexpr int WAVE_N = GEMM_BN / WN;   // columns per wave (rows: 64)
  static constexpr int NJ = WAVE_N / 16;        // MFMA tiles per wave along n (4 along m)
  static GPR_DEV int m0(int wave) { return (wave / WN) * 64; }
  static GPR_DEV int n0(int wave) { return (wave % WN) * WAVE_N; }
};

template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
  typedef v4d acc_t;
  static GPR_DEV acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // f64 16x16x4 output: lane l, register r holds row (l/16) + 4r, column l%16
  static GPR_DEV int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MfmaOp<float> {
  typedef v4f acc_t;
  static GPR_DEV acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // f32 16x16x4 output: lane l, register r holds row 4(l/16) + r, column l%16
  static GPR_DEV int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Per compute type T: K depth of an LDS chunk, elements each thread stages per operand
// and chunk, and LDS row pitch.  16-deep chunks for both float64 and float32 (measured:
// 32-deep float32 chunks, padded float32 pitches and three or four workgroups per CU were
// all slower than two workgroups per CU with this configuration).
template <typename T>
struct Chunk {
  static constexpr int BK = 16;
  static constexpr int LD = GEMM_BM + 4;                   // LDS row pitch (elements)
  static constexpr int SMEM = 2 * 2 * BK * LD * (int)sizeof(T);   // A and B, double-buffered
};
// One thread's share of a chunk operand in a workgroup of Shape<WN>.
template <typename T, int WN>
struct Share {
  static constexpr int E = Chunk<T>::BK * GEMM_BM / Shape<WN>::THREADS;   // 8 or 4 elements
  static constexpr int KPT = 2;                          // KC: consecutive k per thread and row,
  static constexpr int RP = E / KPT;                     //     in RP rows
  static constexpr int RS = Shape<WN>::THREADS / 8;      //     RS apart
  static constexpr int TPR = GEMM_BM / E;                // MC: threads per k row
};
template <typename T>
using LdsBuf = T (*)[Chunk<T>::BK][Chunk<T>::LD];   // [buffer][k][row]
template <typename T>
using LdsChunk = T (*)[Chunk<T>::LD];               // [k][row]

template <typename T>
GPR_DEV void seg_krange(const GemmSeg& s, int m0, int n0, int& kb, int& ke) {
  kb = 0;
  ke = s.K;
  if (s.tri & A_LOWER) ke = min(ke, m0 + GEMM_BM);
  if (s.tri & B_LOWER) ke = min(ke, n0 + GEMM_BN);
  if (s.tri & A_UPPER) kb = max(kb, m0);
  if (s.tri & B_UPPER) kb = max(kb, n0);
  kb = (kb / Chunk<T>::BK) * Chunk<T>::BK;
}

// Operand loads go through global-address-space pointers: generic (flat) loads would
// also count against the LDS wait counter, so waiting for the current chunk's LDS
// fragments would wait for the next chunk's prefetch as well.
template <typename V>
GPR_DEV V load_global(const void* p) {
  typedef __attribute__((address_space(1))) const V gV;
  return *(gV*)(p);
}

// Loads this thread's share of a 128 x BK operand chunk (stored as TL) into registers,
// zero outside [0,lim) x [k0,kend).  KC: KPT consecutive k of RP rows; MC: E consecutive
// rows of one k.  When the whole chunk is in range and the rows are 16-byte aligned (a
// uniform test) the loads are unguarded vector loads; otherwise every element is guarded.
template <typename T, typename TL, int WN>
GPR_DEV void load_chunk(const TL* __restrict__ P, int64_t ld, int mode, int base, int lim, int k0, int kend,
                        int tid, TL (&r)[Share<T, WN>::E]) {
  typedef Share<T, WN> C;
  constexpr int VEC = 16 / sizeof(TL);
  const bool full = ((((uintptr_t)P) & 15) == 0) && ((ld * (int64_t)sizeof(TL)) % 16 == 0) &&
                    base + GEMM_BM <= lim && k0 + Chunk<T>::BK <= kend;
  if (mode == MODE_KC) {
    const int kk = k0 + (tid & 7) * C::KPT;
    if (full) {
      typedef TL vk __attribute__((ext_vector_type(C::KPT)));
#pragma unroll
      for (int p = 0; p < C::RP; ++p) {
        const vk v = load_global<vk>(P + (int64_t)(base + (tid >> 3) + C::RS * p) * ld + kk);
#pragma unroll
        for (int e = 0; e < C::KPT; ++e) r[p * C::KPT + e] = v[e];
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < C::RP; ++p) {
      const int row = base + (tid >> 3) + C::RS * p;
      const bool rok = row < lim;
      const TL* q = P + (int64_t)row * ld + kk;
#pragma unroll
      for (int e = 0; e < C::KPT; ++e) r[p * C::KPT + e] = (rok && kk + e < kend) ? load_global<TL>(q + e) : TL(0);
    }
  } else {
    const int k = k0 + tid / C::TPR;
    const int r0 = base + (tid % C::TPR) * C::E;
    const TL* q = P + (int64_t)k * ld + r0;
    if (full) {
      typedef TL vv __attribute__((ext_vector_type(VEC)));
#pragma unroll
      for (int e = 0; e < C::E; e += VEC) {
        const vv v = load_global<vv>(q + e);
#pragma unroll
        for (int x = 0; x < VEC; ++x) r[e + x] = v[x];
      }
      return;
    }
    const bool kok = k < kend;
#pragma unroll
    for (int e = 0; e < C::E; ++e) r[e] = (kok && r0 + e < lim) ? load_global<TL>(q + e) : TL(0);
  }
}

template <typename T, typename TL, int WN>
GPR_DEV void store_chunk(LdsChunk<T> S, int mode, int tid, const TL (&r)[Share<T, WN>::E]) {
  typedef Share<T, WN> C;
  if (mode == MODE_KC) {
    const int kk = (tid & 7) * C::KPT;
#pragma unroll
    for (int p = 0; p < C::RP; ++p) {
      const int row = (tid >> 3) + C::RS * p;
#pragma unroll
      for (int e = 0; e < C::KPT; ++e) S[kk + e][row] = (T)r[p * C::KPT + e];
    }
  } else {
    const int k = tid / C::TPR;
    const int r0 = (tid % C::TPR) * C::E;
#pragma unroll
    for (int e = 0; e < C::E; ++e) S[k][r0 + e] = (T)r[e];
  }
}

// acc += the products of one LDS chunk: this wave's 64 x WAVE_N block as 4 x NJ MFMA tiles.
template <typename T, int WN>
GPR_DEV void mma_chunk(LdsChunk<T> As, LdsChunk<T> Bs, int lane, int wm, int wn,
                       typename MfmaOp<T>::acc_t (&acc)[4][Shape<WN>::NJ]) {
  constexpr int NJ = Shape<WN>::NJ;
  typedef MfmaOp<T> Op;
#pragma unroll
  for (int kq = 0; kq < Chunk<T>::BK / 4; ++kq) {
    const int kr = kq * 4 + (lane >> 4);
    T a[4], b[NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = Bs[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = Op::mma(a[i], b[j], acc[i][j]);
  }
}

// Finds this workgroup's job and macro tile; returns false when the tile lies above
// the diagonal of a lower-only job.
GPR_DEV bool locate_job(const GemmJob* __restrict__ jobs, int njobs, GemmJob& job, int& m0, int& n0) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_begin <= bid) lo = mid; else hi = mid - 1;
  }
  job = jobs[lo];
  job_tile(job, bid - job.wg_begin, m0, n0);
  return !((job.flags & JOB_LOWER_ONLY) && (m0 + GEMM_BM - 1 < n0));
}

// Guarded main loop (any shapes, alignments and operand modes): acc += sum over the job's
// segments of the 128 x 128 macro tile at (m0, n0).  The next chunk, possibly the first of
// the next segment, is loaded while the current one is multiplied; each load takes the
// vector path when its chunk lies inside an aligned operand.
template <typename T, typename TL, int WN>
GPR_DEV void gemm_mainloop_generic(const GemmJob& job, const GemmSeg* __restrict__ segs, int m0, int n0,
                                   typename MfmaOp<T>::acc_t (&acc)[4][Shape<WN>::NJ], LdsBuf<T> As,
                                   LdsBuf<T> Bs) {
  constexpr int BK = Chunk<T>::BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = Shape<WN>::m0(wave), wn = Shape<WN>::n0(wave);
  const int send = job.seg0 + job.nseg;
  int cs = job.seg0, ck0 = 0, cke = 0;
  for (; cs < send; ++cs) {
    seg_krange<T>(segs[cs], m0, n0, ck0, cke);
    if (ck0 < cke) break;
  }
  if (cs >= send) return;
  TL ra[Share<T, WN>::E], rb[Share<T, WN>::E];
  {
    const GemmSeg& s = segs[cs];
    load_chunk<T, TL, WN>((const TL*)s.A, s.lda, s.modeA, m0, job.M, ck0, cke, tid, ra);
    load_chunk<T, TL, WN>((const TL*)s.B, s.ldb, s.modeB, n0, job.N, ck0, cke, tid, rb);
    store_chunk<T, TL, WN>(As[0], s.modeA, tid, ra);
    store_chunk<T, TL, WN>(Bs[0], s.modeB, tid, rb);
  }
  __syncthreads();
  int buf = 0;
  while (true) {
    int ns = cs, nk0 = ck0 + BK, nke = cke;
    if (nk0 >= cke) {
      for (ns = cs + 1; ns < send; ++ns) {
        seg_krange<T>(segs[ns], m0, n0, nk0, nke);
        if (nk0 < nke) break;
      }
    }
    const bool more = ns < send;
    int nmodeA = 0, nmodeB = 0;
    if (more) {
      const GemmSeg& s = segs[ns];
      nmodeA = s.modeA;
      nmodeB = s.modeB;
      load_chunk<T, TL, WN>((const TL*)s.A, s.lda, s.modeA, m0, job.M, nk0, nke, tid, ra);
      load_chunk<T, TL, WN>((const TL*)s.B, s.ldb, s.modeB, n0, job.N, nk0, nke, tid, rb);
    }
    mma_chunk<T, WN>(As[buf], Bs[buf], lane, wm, wn, acc);
    if (!more) break;
    // keep the stores of the next chunk (which wait for its global loads) after the products
    __builtin_amdgcn_sched_barrier(0);
    store_chunk<T, TL, WN>(As[buf ^ 1], nmodeA, tid, ra);
    store_chunk<T, TL, WN>(Bs[buf ^ 1], nmodeB, tid, rb);
    __syncthreads();
    buf ^= 1;
    cs = ns;
    ck0 = nk0;
    cke = nke;
  }
}

// Unguarded chunk load for a macro tile that lies inside the operand with 16-byte aligned
// rows (the caller has checked); the patterns of load_chunk for a fixed mode.
template <typename T, typename TL, int MODE, int WN>
GPR_DEV void load_chunk_full(const TL* __restrict__ P, int64_t ld, int base, int k0, int tid,
                             TL (&r)[Share<T, WN>::E]) {
  typedef Share<T, WN> C;
  if (MODE == MODE_KC) {
    typedef TL vk __attribute__((ext_vector_type(C::KPT)));
    const int kk = k0 + (tid & 7) * C::KPT;
#pragma unroll
    for (int p = 0; p < C::RP; ++p) {
      const vk v = load_global<vk>(P + (int64_t)(base + (tid >> 3) + C::RS * p) * ld + kk);
#pragma unroll
      for (int e = 0; e < C::KPT; ++e) r[p * C::KPT + e] = v[e];
    }
  } else {
    constexpr int VEC = 16 / sizeof(TL);
    typedef TL vv __attribute__((ext_vector_type(VEC)));
    const TL* q = P + (int64_t)(k0 + tid / C::TPR) * ld + base + (tid % C::TPR) * C::E;
#pragma unroll
    for (int e = 0; e < C::E; e += VEC) {
      const vv v = load_global<vv>(q + e);
#pragma unroll
      for (int x = 0; x < VEC; ++x) r[e + x] = v[x];
    }
  }
}

// One segment's k range [kb, ke) (whole chunks) of a macro tile inside both operands:
// straight-line loads and stores for fixed modes, LDS double buffer, one barrier per chunk.
// Starts with a barrier, so the previous segment's last chunk may still be in LDS.
template <typename T, typename TL, int MA, int MB, int WN>
GPR_DEV void seg_full(const GemmSeg& s, int m0, int n0, int kb, int ke,
                      typename MfmaOp<T>::acc_t (&acc)[4][Shape<WN>::NJ], LdsBuf<T> As, LdsBuf<T> Bs) {
  constexpr int BK = Chunk<T>::BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = Shape<WN>::m0(wave), wn = Shape<WN>::n0(wave);
  const TL* __restrict__ A = (const TL*)s.A;
  const TL* __restrict__ B = (const TL*)s.B;
  TL ra[Share<T, WN>::E], rb[Share<T, WN>::E];
  load_chunk_full<T, TL, MA, WN>(A, s.lda, m0, kb, tid, ra);
  load_chunk_full<T, TL, MB, WN>(B, s.ldb, n0, kb, tid, rb);
  __syncthreads();
  store_chunk<T, TL, WN>(As[0], MA, tid, ra);
  store_chunk<T, TL, WN>(Bs[0], MB, tid, rb);
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 + BK < ke; k0 += BK) {
    load_chunk_full<T, TL, MA, WN>(A, s.lda, m0, k0 + BK, tid, ra);
    load_chunk_full<T, TL, MB, WN>(B, s.ldb, n0, k0 + BK, tid, rb);
    mma_chunk<T, WN>(As[buf], Bs[buf], lane, wm, wn, acc);
    // keep the stores of the next chunk (which wait for its global loads) after the products
    __builtin_amdgcn_sched_barrier(0);
    store_chunk<T, TL, WN>(As[buf ^ 1], MA, tid, ra);
    store_chunk<T, TL, WN>(Bs[buf ^ 1], MB, tid, rb);
    __syncthreads();
    buf ^= 1;
  }
  mma_chunk<T, WN>(As[buf], Bs[buf], lane, wm, wn, acc);
}

// Operand-mode specialisations of the main loop.  SPEC_GUARDED runs the guarded loop; the
// others run the straight-line loop of one operand-mode pair and are chosen by the host
// only for launches whose jobs all cover whole macro tiles (M, N multiples of 128), whose
// segments all have K a multiple of the chunk depth, 16-byte aligned rows and that pair.
enum { SPEC_GUARDED = -1, SPEC_KK = 0, SPEC_KM = 1, SPEC_MM = 3 };

template <typename T, typename TL, int SPEC, int WN>
GPR_DEV void gemm_mainloop(const GemmJob& job, const GemmSeg* __restrict__ segs, int m0, int n0,
                           typename MfmaOp<T>::acc_t (&acc)[4][Shape<WN>::NJ], LdsBuf<T> As, LdsBuf<T> Bs) {
  if constexpr (SPEC == SPEC_GUARDED) {
    gemm_mainloop_generic<T, TL, WN>(job, segs, m0, n0, acc, As, Bs);
  } else {
    for (int cs = job.seg0; cs < job.seg0 + job.nseg; ++cs) {
      const GemmSeg& s = segs[cs];
      int kb, ke;
      seg_krange<T>(s, m0, n0, kb, ke);
      if (kb < ke) seg_full<T, TL, (SPEC >> 1), (SPEC & 1), WN>(s, m0, n0, kb, ke, acc, As, Bs);
    }
  }
}

// One macro tile (m0, n0) of `job`: the products of its segments, then the epilogue
// C = alpha * acc + beta * Cin.  smem: Chunk<T>::SMEM bytes of LDS.
template <typename T, typename TL, int SPEC, int WN>
GPR_DEV void gemm_tile_work(const GemmJob& job, const GemmSeg* __restrict__ segs, int m0, int n0, char* smem) {
  typedef MfmaOp<T> Op;
  typedef typename Op::acc_t acc_t;
  constexpr int NJ = Shape<WN>::NJ;
  LdsBuf<T> As = reinterpret_cast<LdsBuf<T>>(smem);
  LdsBuf<T> Bs = As + 2;
  acc_t acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  gemm_mainloop<T, TL, SPEC, WN>(job, segs, m0, n0, acc, As, Bs);

  // epilogue: C = alpha * acc + beta * Cin
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = Shape<WN>::m0(wave), wn = Shape<WN>::n0(wave);
  const bool c32 = job.flags & JOB_C_F32;
  const double alpha = job.alpha, beta = job.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + Op::row(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < job.M && col < job.N) {
          double v = alpha * (double)acc[i][j][r];
          if (c32) {
            if (beta != 0.0) v += beta * (double)((const float*)job.Cin)[(int64_t)row * job.ldcin + col];
            ((float*)job.C)[(int64_t)row * job.ldc + col] = (float)v;
          } else {
            if (beta != 0.0) v += beta * ((const double*)job.Cin)[(int64_t)row * job.ldcin + col];
            ((double*)job.C)[(int64_t)row * job.ldc + col] = v;
          }
        }
      }
}

template <typename T, typename TL, int SPEC, int WN>
GPR_DEV void gemm_tiles_body(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  __shared__ __align__(16) char smem[Chunk<T>::SMEM];
  GemmJob job;
  int m0, n0;
  if (!locate_job(jobs, njobs, job, m0, n0)) return;
  gemm_tile_work<T, TL, SPEC, WN>(job, segs, m0, n0, smem);
}

}  // namespace gpr
