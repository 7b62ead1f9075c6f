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

}  // namespace gpr
