// Trailing update with split-BF16 products on the gfx950 matrix cores.
//
// After the panel solve, every float32 panel element x is split into three
// bfloat16 parts hi + mid + lo (round to nearest even at each step; the two
// residual subtractions are exact in float32).  The update A_mn -= A_mk A_nk^T
// then sums the bfloat16 products with float32 accumulation on
// v_mfma_f32_16x16x32_bf16: hh + hm + mh (bf16x3, about 16 significant bits) or
// additionally hl + lh + mm (bf16x6, close to float32), issuing the small products
// first within each 32-deep step.  A 256-thread workgroup computes a 128 x 128
// macro tile; each wave64 owns a 64 x 64 quadrant as 4 x 4 accumulators.  The
// planes are staged k-contiguous in LDS with an 80-byte row pitch, so one
// 16-byte fragment read by 16 lanes covers all 64 banks once.
#include "common.h"
#include "kernels.h"

namespace gpr {

constexpr int BF_BK = 32;                 // k per chunk (one MFMA k-step)
constexpr int BF_PITCH = BF_BK + 8;       // bf16 elements per LDS row (80 bytes)

typedef unsigned short bfraw;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 8 packed bfloat16

GPR_DEV bfraw bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bfraw)((u >> 16) | 0x40);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bfraw)(u >> 16);
}
GPR_DEV float bf16_to_float(bfraw h) { return __uint_as_float(((uint32_t)h) << 16); }

// hi + mid + lo of float32 x
__global__ void split_bf16x3_kernel(const float* __restrict__ x, int64_t count, bfraw* __restrict__ hi,
                                   bfraw* __restrict__ mid, bfraw* __restrict__ lo) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = x[i];
    const bfraw h = bf16_rne_bits(v);
    const float r1 = v - bf16_to_float(h);
    const bfraw m = bf16_rne_bits(r1);
    const float r2 = r1 - bf16_to_float(m);
    hi[i] = h;
    mid[i] = m;
    if (lo) lo[i] = bf16_rne_bits(r2);
  }
}

// Loads this thread's share (one row, 16 consecutive k) of a 128 x 32 chunk of one plane.
// When the whole chunk lies inside the plane with 16-byte aligned rows (a test that is
// uniform over the workgroup) the loads are unguarded vector loads; otherwise every
// element is guarded.  The loads go through global-address-space pointers: generic
// (flat) loads would also count against the LDS wait counter, so the waits for the LDS
// fragments of the current chunk would wait for the next chunk's loads as well.
GPR_DEV void bf_load(const bfraw* __restrict__ P, int64_t ld, int base, int lim, int k0, int kend, int tid,
                     u32x4& r0, u32x4& r1) {
  typedef __attribute__((address_space(1))) const u32x4 gu4;
  typedef __attribute__((address_space(1))) const bfraw gbf;
  const bool full = ((((uintptr_t)P) & 15) == 0) && ((ld * (int64_t)sizeof(bfraw)) % 16 == 0) &&
                    base + GEMM_BM <= lim && k0 + BF_BK <= kend;
  const int row = base + (tid >> 1);
  const int kk = k0 + (tid & 1) * 16;
  const bfraw* q = P + (int64_t)row * ld + kk;
  if (full) {
    r0 = *(gu4*)q;
    r1 = *(gu4*)(q + 8);
  } else {
    bfraw t[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = (row < lim && kk + e < kend) ? *(gbf*)(q + e) : (bfraw)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      r0[e] = (unsigned)t[2 * e] | ((unsigned)t[2 * e + 1] << 16);
      r1[e] = (unsigned)t[8 + 2 * e] | ((unsigned)t[8 + 2 * e + 1] << 16);
    }
  }
}

template <int NPLANES>
GPR_DEV void bf_store(bfraw* S, int tid, const u32x4 (&r)[NPLANES][2]) {
  const int row = tid >> 1, kk = (tid & 1) * 16;
#pragma unroll
  for (int p = 0; p < NPLANES; ++p) {
    u32x4* d = (u32x4*)(S + (p * GEMM_BM + row) * BF_PITCH + kk);
    d[0] = r[p][0];
    d[1] = r[p][1];
  }
}

GPR_DEV v8bf frag(const bfraw* S, int plane, int row, int koff) {
  const uint4 v = *(const uint4*)(S + (plane * GEMM_BM + row) * BF_PITCH + koff);
  return __builtin_bit_cast(v8bf, v);
}

GPR_DEV v4f mma_bf16(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// NPROD = 3 (hh, hm, mh) or 6 (+ hl, lh, mm).  Operands are MODE_KC with no triangular skips.
template <int NPROD>
__global__ __launch_bounds__(GEMM_THREADS, 2)
void gemm_bf16x_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  constexpr int NP = NPROD == 6 ? 3 : 2;   // planes needed
  __shared__ __align__(16) bfraw As[NP * GEMM_BM * BF_PITCH];
  __shared__ __align__(16) bfraw Bs[NP * GEMM_BN * BF_PITCH];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_begin <= bid) lo = mid; else hi = mid - 1;
  }
  const GemmJob job = jobs[lo];
  int m0, n0;
  job_tile(job, bid - job.wg_begin, m0, n0);
  if ((job.flags & JOB_LOWER_ONLY) && (m0 + GEMM_BM - 1 < n0)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  // Chunks (segment, k0) in order; the next chunk's planes are loaded into registers
  // while the current one is multiplied from LDS (two barriers per chunk; the planes of
  // one chunk take 60 KB of LDS, so two workgroups share a CU).
  const int send = job.seg0 + job.nseg;
  int s = job.seg0;
  while (s < send && segs[s].K <= 0) ++s;
  if (s < send) {
    const int koff = (lane >> 4) * 8;
    u32x4 ra[NP][2], rb[NP][2];
    int k0 = 0;
    auto load = [&](int si, int kk) {
      const GemmSeg& sg = segs[si];
      const bfraw* A = (const bfraw*)sg.A;
      const bfraw* B = (const bfraw*)sg.B;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        bf_load(A + p * sg.pstrideA, sg.lda, m0, job.M, kk, sg.K, tid, ra[p][0], ra[p][1]);
        bf_load(B + p * sg.pstrideB, sg.ldb, n0, job.N, kk, sg.K, tid, rb[p][0], rb[p][1]);
      }
    };
    load(s, k0);
    while (true) {
      __syncthreads();   // previous chunk fully consumed
      bf_store<NP>(As, tid, ra);
      bf_store<NP>(Bs, tid, rb);
      __syncthreads();
      int ns = s, nk0 = k0 + BF_BK;
      if (nk0 >= segs[s].K) {
        nk0 = 0;
        for (ns = s + 1; ns < send && segs[ns].K <= 0; ++ns) {
        }
      }
      const bool more = ns < send;
      if (more) load(ns, nk0);
      v8bf a[4][NP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int p = 0; p < NP; ++p) a[i][p] = frag(As, p, wm + i * 16 + (lane & 15), koff);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v8bf b[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) b[p] = frag(Bs, p, wn + j * 16 + (lane & 15), koff);
        // small products first: (mm, lh, hl), then (mh, hm), then hh
        if (NPROD == 6) {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][1], b[1], acc[i][j]);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][2 % NP], b[0], acc[i][j]);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][0], b[2 % NP], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][1], b[0], acc[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][0], b[1], acc[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf16(a[i][0], b[0], acc[i][j]);
      }
      if (!more) break;
      s = ns;
      k0 = nk0;
    }
  }

  const bool c32 = job.flags & JOB_C_F32;
  const double alpha = job.alpha, beta = job.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
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

hipError_t launch_gemm_bf16(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg, hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (nprod == 6)
    hipLaunchKernelGGL(gemm_bf16x_kernel<6>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
  else
    hipLaunchKernelGGL(gemm_bf16x_kernel<3>, dim3(nwg), dim3(GEMM_THREADS), 0, st, jobs, segs, njobs);
  return hipGetLastError();
}

hipError_t launch_split_bf16x3(const float* x, int64_t count, void* hi, void* mid, void* lo, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(split_bf16x3_kernel, dim3((unsigned)g), dim3(256), 0, st, x, count, (bfraw*)hi, (bfraw*)mid,
                     (bfraw*)lo);
  return hipGetLastError();
}


// ---------------------------------------------------------------- 256 x 256 macro tiles
//
// The trailing update of tiles whose edge is a multiple of 256 uses planes in a tiled
// layout and a larger macro tile.  Within each b x b tile of a plane, element (r, c) is at
//   ((r / 256) (b / 16) + c / 16) 4096 + (r % 256) 16 + c % 16,
// so a 256-row x 16-deep chunk is 8 KB of contiguous memory (fully coalesced loads; each
// tile still occupies its b^2 elements, at the same offset as in the row-major layout).
// A 512-thread workgroup (eight wave64s as 2 x 4, each 128 x 64) computes a 256 x 256
// macro tile with v_mfma_f32_32x32x16_bf16 (4 x 2 accumulators of 32 x 32 per wave).
// Chunks are 16 deep and double-buffered in LDS, one barrier per chunk.  LDS rows are 48
// bytes (the 32 bytes of a chunk row and 16 of padding): the 16-byte fragment reads of
// 16 consecutive lanes (rows r..r+15) then fall on 16 distinct 16-byte bank groups (with
// unpadded 32-byte rows the counters showed bank conflicts on 37 % of the LDS cycles).  The planes of chunk c+2 are loaded into registers (a ring of two)
// while chunk c is multiplied, so each load has two chunks' products to arrive: with one
// workgroup per CU a single chunk of look-ahead left the matrix cores waiting on L2.
// Against the 128 x 128 tiles above this halves the operand bytes per product fetched
// from L2 and cuts the LDS fragment reads per product by a quarter.
constexpr int BT_M = 256;                 // macro tile edge
constexpr int BT_K = 16;                  // chunk depth
constexpr int BT_PITCH = 24;              // bf16 elements per LDS row (48 bytes)
constexpr int BT_THREADS = 512;

typedef float v16f __attribute__((ext_vector_type(16)));

GPR_DEV v16f mma32_bf16(v8bf a, v8bf b, v16f c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }

// hi + mid (+ lo) of float32 x, written in the tiled layout (tiles of edge b, b % 256 == 0).
// Thread i produces output element i of each plane: element (r, c) of the source.
__global__ void split_bf16x3_tiled_kernel(const float* __restrict__ x, int64_t count, int64_t b,
                                          bfraw* __restrict__ hi, bfraw* __restrict__ mid, bfraw* __restrict__ lo) {
  const int64_t bb = b * b, kc = b / BT_K;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < count; o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = o / bb, rem = o % bb;
    const int64_t blk = rem >> 12, within = rem & 4095;
    const int64_t r = q * b + (blk / kc) * BT_M + (within >> 4);
    const int64_t c = (blk % kc) * BT_K + (within & 15);
    const float v = x[r * b + c];
    const bfraw h = bf16_rne_bits(v);
    const float r1 = v - bf16_to_float(h);
    const bfraw m = bf16_rne_bits(r1);
    const float r2 = r1 - bf16_to_float(m);
    hi[o] = h;
    mid[o] = m;
    if (lo) lo[o] = bf16_rne_bits(r2);
  }
}

template <int NP>
struct BtRegs {
  u32x4 a[NP], b[NP];
};

// This thread's 16 bytes of each plane of the chunk (row tid / 2, k half tid % 2).
template <int NP>
GPR_DEV void bt_load(const bfraw* A, const bfraw* B, int64_t pa, int64_t pb, int64_t offa, int64_t offb, int tid,
                     BtRegs<NP>& r) {
  typedef __attribute__((address_space(1))) const u32x4 gu4;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    r.a[p] = *(gu4*)(A + p * pa + offa + tid * 8);
    r.b[p] = *(gu4*)(B + p * pb + offb + tid * 8);
  }
}

template <int NP>
GPR_DEV void bt_store(bfraw* As, bfraw* Bs, int tid, const BtRegs<NP>& r) {
  const int off = (tid >> 1) * BT_PITCH + (tid & 1) * 8;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    *(u32x4*)(As + p * BT_M * BT_PITCH + off) = r.a[p];
    *(u32x4*)(Bs + p * BT_M * BT_PITCH + off) = r.b[p];
  }
}

GPR_DEV v8bf bt_frag(const bfraw* S, int plane, int row, int koff) {
  const uint4 v = *(const uint4*)(S + (plane * BT_M + row) * BT_PITCH + koff);
  return __builtin_bit_cast(v8bf, v);
}

// acc += the products of one LDS chunk (this wave's 128 x 64 block).  Rows are taken two
// 32-row blocks at a time and each product type is issued for the four accumulators of
// the pair before the next, so that consecutive matrix-core instructions do not depend on
// each other.
template <int NPROD, int NP>
GPR_DEV void bt_mma(const bfraw* As, const bfraw* Bs, int wm, int wn, int frow, int fk, v16f (&acc)[4][2]) {
  v8bf b[2][NP];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int p = 0; p < NP; ++p) b[j][p] = bt_frag(Bs, p, wn + j * 32 + frow, fk);
#pragma unroll
  for (int i0 = 0; i0 < 4; i0 += 2) {
    v8bf a[2][NP];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int p = 0; p < NP; ++p) a[ii][p] = bt_frag(As, p, wm + (i0 + ii) * 32 + frow, fk);
    // plane pairs (A, B), small products first: (mm, lh, hl), then (mh, hm), then hh
    constexpr int NQ = NPROD == 6 ? 6 : 3;
    constexpr int PA[6] = {1, 2, 0, 1, 0, 0}, PB[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
    for (int q = (NPROD == 6 ? 0 : 3); q < 6; ++q)
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i0 + ii][j] = mma32_bf16(a[ii][PA[q] % NP], b[j][PB[q] % NP], acc[i0 + ii][j]);
    (void)NQ;
  }
}

// Job and macro tile of workgroup `bid` of a 256 x 256 launch: the job whose workgroup
// range holds bid, its macro tiles in 8 x 8 patches when both grid extents are multiples
// of 8, row-major otherwise.
GPR_DEV void t256_locate(const GemmJob* __restrict__ jobs, int njobs, int bid, GemmJob& job, int& m0, int& n0) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int midj = (lo + hi + 1) >> 1;
    if (jobs[midj].wg_begin <= bid) lo = midj; else hi = midj - 1;
  }
  job = jobs[lo];
  const int t = bid - job.wg_begin, tn = job.tiles_n, tm = job.M / BT_M;
  if ((tn & 7) == 0 && (tm & 7) == 0) {
    const int sb = t >> 6, w = t & 63, sbn = tn >> 3;
    m0 = ((sb / sbn) * 8 + (w >> 3)) * BT_M;
    n0 = ((sb % sbn) * 8 + (w & 7)) * BT_M;
  } else {
    m0 = (t / tn) * BT_M;
    n0 = (t % tn) * BT_M;
  }
}

template <int NPROD>
struct T256 {
  static constexpr int NP = NPROD == 6 ? 3 : 2;
  static constexpr int HALF = NP * BT_M * BT_PITCH;   // the A (then the B) planes of one chunk
  static constexpr int SMEM = 2 * 2 * HALF;           // bfloat16 elements of LDS, double-buffered
};

// acc = the split-bfloat16 products of every segment of the job for the macro tile at
// (m0, n0): wave `wave` owns rows wm .. wm+127 and columns wn .. wn+63 as 4 x 2
// accumulators of 32 x 32.  smem: T256<NPROD>::SMEM elements.
template <int NPROD>
GPR_DEV void t256_mainloop(const GemmJob& job, const GemmSeg* __restrict__ segs, int m0, int n0, bfraw* smem,
                           v16f (&acc)[4][2], int tid, int wm, int wn, int frow, int fk) {
  constexpr int NP = T256<NPROD>::NP;
  constexpr int HALF = T256<NPROD>::HALF;
  bfraw* const L0 = smem;              // chunk buffer 0: A planes, then B planes
  bfraw* const L1 = smem + 2 * HALF;   // chunk buffer 1
  bool primed = false;
  for (int s = job.seg0; s < job.seg0 + job.nseg; ++s) {
    const GemmSeg& sg = segs[s];
    const int nck = sg.K / BT_K;
    if (nck <= 0) continue;
    const bfraw* A = (const bfraw*)sg.A;
    const bfraw* B = (const bfraw*)sg.B;
    const int64_t pa = sg.pstrideA, pb = sg.pstrideB;
    // offsets of the macro tile's 256-row blocks: chunk c is at + c 4096
    const int64_t offa = (int64_t)(m0 / BT_M) * (sg.lda / BT_K) * 4096;
    const int64_t offb = (int64_t)(n0 / BT_M) * (sg.ldb / BT_K) * 4096;
    // chunk q lives in registers r[q % 2] until it is stored into LDS buffer q % 2.  The
    // loads are issued unconditionally -- past the last chunk they re-read the last one,
    // which is then never stored -- and kept ahead of the products by a scheduling
    // barrier: with a load under a condition the compiler waited for every load in
    // flight before each store into LDS and sank the loads below the products (measured:
    // +3.5 % bf16x6, +4.4 % bf16x3 on the trailing update).
    const int64_t last = (int64_t)(nck - 1) * 4096;
    auto chunk_at = [&](int q) { return q < nck ? (int64_t)q * 4096 : last; };
    BtRegs<NP> r0, r1;
    bt_load<NP>(A, B, pa, pb, offa, offb, tid, r0);
    bt_load<NP>(A, B, pa, pb, offa + chunk_at(1), offb + chunk_at(1), tid, r1);
    if (primed) __syncthreads();   // the previous segment's last chunk has been read
    bt_store<NP>(L0, L0 + HALF, tid, r0);
    __syncthreads();
    primed = true;
    for (int c = 0; c < nck; c += 2) {
      // even chunk c from buffer 0; chunk c+1 waits in r1, chunk c+2 is loaded into r0
      bt_load<NP>(A, B, pa, pb, offa + chunk_at(c + 2), offb + chunk_at(c + 2), tid, r0);
      __builtin_amdgcn_sched_barrier(0);
      bt_mma<NPROD, NP>(L0, L0 + HALF, wm, wn, frow, fk, acc);
      if (c + 1 >= nck) break;
      __builtin_amdgcn_sched_barrier(0);
      bt_store<NP>(L1, L1 + HALF, tid, r1);
      __syncthreads();
      // odd chunk c+1 from buffer 1; chunk c+2 waits in r0, chunk c+3 is loaded into r1
      bt_load<NP>(A, B, pa, pb, offa + chunk_at(c + 3), offb + chunk_at(c + 3), tid, r1);
      __builtin_amdgcn_sched_barrier(0);
      bt_mma<NPROD, NP>(L1, L1 + HALF, wm, wn, frow, fk, acc);
      if (c + 2 >= nck) break;
      __builtin_amdgcn_sched_barrier(0);
      bt_store<NP>(L0, L0 + HALF, tid, r0);
      __syncthreads();
    }
  }
}

// 32 x 32 float32 accumulator layout: lane l, register r holds column l % 32 and row
// 8 (r / 4) + 4 (l / 32) + r % 4 of its block
GPR_DEV int t256_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// C = alpha * (products) + beta * Cin for each job of whole 256 x 256 macro tiles.
template <int NPROD>
GPR_DEV void t256_body(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs, bfraw* smem) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  GemmJob job;
  int m0, n0;
  t256_locate(jobs, njobs, bid, job, m0, n0);
  if ((job.flags & JOB_LOWER_ONLY) && (m0 + BT_M - 1 < n0)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
  const int frow = lane & 31, fk = (lane >> 5) * 8;

  v16f acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  t256_mainloop<NPROD>(job, segs, m0, n0, smem, acc, tid, wm, wn, frow, fk);

  const bool c32 = job.flags & JOB_C_F32;
  const double alpha = job.alpha, beta = job.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + i * 32 + t256_row(lane, r);
        const int col = n0 + wn + j * 32 + (lane & 31);
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

// NPROD = 3 (hh, hm, mh) or 6 (+ hl, lh, mm).  Every job covers whole 256 x 256 macro
// tiles, every segment is a pair of tiled-layout planes (lda = ldb = K, a multiple of 16,
// no triangular skips); the host checks this before the launch.
template <int NPROD>
__global__ __launch_bounds__(BT_THREADS, 1)
void gemm_bf16x_t256_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  __shared__ __align__(16) bfraw smem[T256<NPROD>::SMEM];
  t256_body<NPROD>(jobs, segs, njobs, smem);
}

// Steps of the triangular inversion L^{-1} of the gradient from split-bfloat16 planes
// (same code as the update, its own symbol).
template <int NPROD>
__global__ __launch_bounds__(BT_THREADS, 1)
void gemm_bf16x_trtri_t256_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  __shared__ __align__(16) bfraw smem[T256<NPROD>::SMEM];
  t256_body<NPROD>(jobs, segs, njobs, smem);
}

// The gradient reduction fused into the K^{-1} products (as gemm_trace_kernel in
// gemm.hip, on 256 x 256 macro tiles of split-bfloat16 products): each job is the
// contribution X_ki^T X_kj of block row k of X = L^{-1} to the K^{-1} tile (i, j) = (aux0,
// aux1); every element w of it (less alpha_r alpha_c when the job carries JOB_TRACE_ALPHA)
// is weighted with the kernel value and its derivative with respect to log l at the tile
// pair's u = r^2 / (2 l^2), and the workgroup writes the sums (sum w dk/dlog l, sum w k,
// sum over the diagonal of w) to partial[blockIdx.x][0..2].  A diagonal tile pair
// (JOB_LOWER_ONLY) runs the macro tiles on and below its diagonal; its strictly-lower
// entries count twice, as do all entries of an off-diagonal pair.  Skipped macro tiles
// write zeros.
template <int NPROD>
__global__ __launch_bounds__(BT_THREADS, 1)
void gemm_bf16x_trace_t256_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs,
                                  TraceArgs ta) {
  __shared__ __align__(16) bfraw smem[T256<NPROD>::SMEM];
  __shared__ double red[3][BT_THREADS / 64];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  GemmJob job;
  int m0, n0;
  t256_locate(jobs, njobs, bid, job, m0, n0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
  const int frow = lane & 31, fk = (lane >> 5) * 8;
  double s_l = 0.0, s_nu = 0.0, s_s = 0.0;
  if (!((job.flags & JOB_LOWER_ONLY) && (m0 + BT_M - 1 < n0))) {
    v16f acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    t256_mainloop<NPROD>(job, segs, m0, n0, smem, acc, tid, wm, wn, frow, fk);
    double ell, nu, s2;
    resolve_hyper(ta.h, ell, nu, s2);
    const int64_t ti = job.aux0, tj = job.aux1;
    const bool diag_tile = ti == tj;
    const bool with_alpha = job.flags & JOB_TRACE_ALPHA;
    const double* __restrict__ U = ta.u + (ti * (ti + 1) / 2 + tj) * ta.b * ta.b;
    if (ta.h.kernel == KERNEL_SE) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = m0 + wm + i * 32 + t256_row(lane, r);
            const int col = n0 + wn + j * 32 + (lane & 31);
            const double wt = !diag_tile || row > col ? 2.0 : (row == col ? 1.0 : 0.0);
            if (wt != 0.0) {
              const double u = U[(int64_t)row * ta.b + col];
              double w = (double)acc[i][j][r];
              if (with_alpha) w -= ta.alpha[ti * ta.b + row] * ta.alpha[tj * ta.b + col];
              const double kf = nu * exp(-u);
              s_l = fma(wt * w * kf, 2.0 * u, s_l);
              s_nu = fma(wt * w, kf, s_nu);
              if (diag_tile && row == col) s_s += w;
            }
          }
    } else {
      // The Matern weights are too long a body to unroll 128 times: each lane parks 32 of
      // its accumulators at a time in its own LDS slots (free once every wave has left the
      // main loop) and walks them in a loop.
      __syncthreads();
      float* const stage = reinterpret_cast<float*>(smem) + wave * 32 * 64;
      const int kern = ta.h.kernel;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) stage[(j * 16 + r) * 64 + lane] = acc[i][j][r];
        for (int q = 0; q < 32; ++q) {
          const int row = m0 + wm + i * 32 + t256_row(lane, q & 15);
          const int col = n0 + wn + (q >> 4) * 32 + (lane & 31);
          const double wt = !diag_tile || row > col ? 2.0 : (row == col ? 1.0 : 0.0);
          if (wt != 0.0) {
            const double u = U[(int64_t)row * ta.b + col];
            double w = (double)stage[q * 64 + lane];
            if (with_alpha) w -= ta.alpha[ti * ta.b + row] * ta.alpha[tj * ta.b + col];
            double kf, dl;
            matern_and_dlogl(kern, u, nu, kf, dl);
            s_l = fma(wt * w, dl, s_l);
            s_nu = fma(wt * w, kf, s_nu);
            if (diag_tile && row == col) s_s += w;
          }
        }
      }
    }
  }
  // fixed-order reduction: butterfly within each wave, then the eight wave sums in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s_l += __shfl_xor(s_l, o);
    s_nu += __shfl_xor(s_nu, o);
    s_s += __shfl_xor(s_s, o);
  }
  if (lane == 0) {
    red[0][wave] = s_l;
    red[1][wave] = s_nu;
    red[2][wave] = s_s;
  }
  __syncthreads();
  if (tid < 3) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < BT_THREADS / 64; ++q) t += red[tid][q];
    ta.partial[(int64_t)blockIdx.x * 3 + tid] = t;
  }
}

// Split-bfloat16 planes of up to 32 float32 blocks given by address, each a rows x kd
// operand (rows and kd multiples of 256 and 16) read from a row-major source with
// leading dimension ld -- element (r, c) at src[r ld + c], or at src[c ld + r] (TRANS: the
// operand is the transpose of a kd x rows source block) -- written in the tiled layout
// above: block t at out + t rows kd of each plane (plane stride pstride elements).
// Workgroup (x, t): the 256 x 16 chunk x of block t, one thread per operand row (reading
// 16 elements of a source row, or of a source column: consecutive threads read
// consecutive addresses), 32 bytes written per plane.  lo is written when np == 3.
struct TileList {
  const float* p[32];
};
template <bool TRANS>
__global__ __launch_bounds__(256)
void split_bf16_tiles_kernel(TileList list, int64_t rows, int64_t kd, int64_t ld, bfraw* __restrict__ out,
                             int64_t pstride, int np) {
  const int64_t t = blockIdx.y, kc = kd / BT_K;
  const int64_t rb = blockIdx.x / kc, kb = blockIdx.x % kc;
  const int64_t r = rb * BT_M + threadIdx.x;   // operand row
  const float* __restrict__ src = list.p[t];
  float x[16];
  if (TRANS) {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = src[(kb * BT_K + e) * ld + r];
  } else {
    const float4* q = (const float4*)(src + r * ld + kb * BT_K);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float4 f = q[e];
      x[4 * e] = f.x;
      x[4 * e + 1] = f.y;
      x[4 * e + 2] = f.z;
      x[4 * e + 3] = f.w;
    }
  }
  unsigned hw[8], mw[8], lw[8];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float v = x[e];
    const bfraw h = bf16_rne_bits(v);
    const float r1 = v - bf16_to_float(h);
    const bfraw m = bf16_rne_bits(r1);
    const bfraw l = bf16_rne_bits(r1 - bf16_to_float(m));
    if (e & 1) {
      hw[e >> 1] |= (unsigned)h << 16;
      mw[e >> 1] |= (unsigned)m << 16;
      lw[e >> 1] |= (unsigned)l << 16;
    } else {
      hw[e >> 1] = h;
      mw[e >> 1] = m;
      lw[e >> 1] = l;
    }
  }
  const int64_t o = t * rows * kd + blockIdx.x * 4096 + (int64_t)threadIdx.x * 16;
  u32x4* dh = (u32x4*)(out + o);
  u32x4* dm = (u32x4*)(out + pstride + o);
  dh[0] = u32x4{hw[0], hw[1], hw[2], hw[3]};
  dh[1] = u32x4{hw[4], hw[5], hw[6], hw[7]};
  dm[0] = u32x4{mw[0], mw[1], mw[2], mw[3]};
  dm[1] = u32x4{mw[4], mw[5], mw[6], mw[7]};
  if (np == 3) {
    u32x4* dl = (u32x4*)(out + 2 * pstride + o);
    dl[0] = u32x4{lw[0], lw[1], lw[2], lw[3]};
    dl[1] = u32x4{lw[4], lw[5], lw[6], lw[7]};
  }
}

// The forward substitution of the posterior variance (V_i = W_ii (B_i - sum_j L_ij V_j))
// from split-bfloat16 planes (same code as the update, its own symbol).
template <int NPROD>
__global__ __launch_bounds__(BT_THREADS, 1)
void gemm_bf16x_solve_t256_kernel(const GemmJob* __restrict__ jobs, const GemmSeg* __restrict__ segs, int njobs) {
  __shared__ __align__(16) bfraw smem[T256<NPROD>::SMEM];
  t256_body<NPROD>(jobs, segs, njobs, smem);
}

hipError_t launch_gemm_bf16_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                 hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (nprod == 6)
    hipLaunchKernelGGL(gemm_bf16x_t256_kernel<6>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  else
    hipLaunchKernelGGL(gemm_bf16x_t256_kernel<3>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_trtri_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (nprod == 6)
    hipLaunchKernelGGL(gemm_bf16x_trtri_t256_kernel<6>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  else
    hipLaunchKernelGGL(gemm_bf16x_trtri_t256_kernel<3>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_trace_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       const TraceArgs& ta, hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (nprod == 6)
    hipLaunchKernelGGL(gemm_bf16x_trace_t256_kernel<6>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs, ta);
  else
    hipLaunchKernelGGL(gemm_bf16x_trace_t256_kernel<3>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs, ta);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_solve_t256(int nprod, const GemmJob* jobs, const GemmSeg* segs, int njobs, int nwg,
                                       hipStream_t st) {
  if (nwg <= 0 || njobs <= 0) return hipSuccess;
  if (nprod == 6)
    hipLaunchKernelGGL(gemm_bf16x_solve_t256_kernel<6>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  else
    hipLaunchKernelGGL(gemm_bf16x_solve_t256_kernel<3>, dim3(nwg), dim3(BT_THREADS), 0, st, jobs, segs, njobs);
  return hipGetLastError();
}

hipError_t launch_split_bf16_tiles(const float* const* blocks, int64_t nblocks, int64_t rows, int64_t kd, int64_t ld,
                                   bool trans, void* out, int64_t pstride, int np, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (rows % BT_M != 0 || kd % BT_K != 0 || rows <= 0 || kd <= 0 || (np != 2 && np != 3) ||
      (((uintptr_t)out) & 15) != 0 || pstride % 8 != 0 || (!trans && ld % 4 != 0) || ld < (trans ? rows : kd))
    return hipErrorInvalidValue;
  for (int64_t t = 0; t < nblocks; ++t)
    if (((uintptr_t)blocks[t]) & 15) return hipErrorInvalidValue;
  for (int64_t t0 = 0; t0 < nblocks; t0 += 32) {
    const int64_t nt = nblocks - t0 < 32 ? nblocks - t0 : 32;
    TileList list{};
    for (int64_t t = 0; t < nt; ++t) list.p[t] = blocks[t0 + t];
    bfraw* o = (bfraw*)out + t0 * rows * kd;
    const dim3 grid((unsigned)((rows / BT_M) * (kd / BT_K)), (unsigned)nt);
    if (trans)
      hipLaunchKernelGGL(split_bf16_tiles_kernel<true>, grid, dim3(256), 0, st, list, rows, kd, ld, o, pstride, np);
    else
      hipLaunchKernelGGL(split_bf16_tiles_kernel<false>, grid, dim3(256), 0, st, list, rows, kd, ld, o, pstride, np);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_split_bf16x3_tiled(const float* x, int64_t count, int64_t b, void* hi, void* mid, void* lo,
                                     hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (b % BT_M != 0 || count % (b * b) != 0) return hipErrorInvalidValue;
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(split_bf16x3_tiled_kernel, dim3((unsigned)g), dim3(256), 0, st, x, count, b, (bfraw*)hi,
                     (bfraw*)mid, (bfraw*)lo);
  return hipGetLastError();
}

}  // namespace gpr
