// Learned warm start: dataset summary statistics and the 32-128-128-3 GELU network.
//
// Statistics (float64, one workgroup): quantiles of the per-feature variances of
// the raw features, quantiles of the log pairwise distances over a given
// subsample of the standardised features (bitonic sort in the workspace), and the
// log variance of the raw targets.  Quantiles interpolate linearly between order
// statistics at position q (count - 1).
//
// Network (float32, one fused workgroup): forward pass of a batch, mean-squared
// error, backward pass and an Adam update of all 21,123 parameters, with every
// reduction in a fixed order so that training is bitwise reproducible.
#include "common.h"
#include "kernels.h"

namespace gpr {

// ---------------------------------------------------------------- statistics
constexpr int ST_THREADS = 1024;

GPR_DEV double quantile_sorted(const double* xs, int64_t cnt, double q) {
  const double h = q * (double)(cnt - 1);
  int64_t lo = (int64_t)floor(h);
  if (lo < 0) lo = 0;
  if (lo > cnt - 1) lo = cnt - 1;
  const int64_t hi = lo + 1 < cnt ? lo + 1 : cnt - 1;
  return xs[lo] + (h - (double)lo) * (xs[hi] - xs[lo]);
}

// ascending bitonic sort of buf[0..len), len a power of two, by the whole workgroup
GPR_DEV void bitonic_sort(double* buf, int64_t len) {
  for (int64_t k = 2; k <= len; k <<= 1) {
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
        const int64_t p = i ^ j;
        if (p > i) {
          const double a = buf[i], b = buf[p];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            buf[i] = b;
            buf[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(ST_THREADS)
void summary_stats_kernel(const double* __restrict__ Zraw, const double* __restrict__ Zstd,
                          const double* __restrict__ yraw, int64_t n, int64_t d, const int64_t* __restrict__ sub,
                          int64_t nsub, double* __restrict__ work, int64_t len, double* __restrict__ out64,
                          float* __restrict__ out32) {
  __shared__ double var[256];
  __shared__ double red[ST_THREADS];
  __shared__ double res[32];
  const int tid = threadIdx.x;
  // per-feature population variance of the raw features (two passes)
  for (int64_t f = tid; f < d; f += ST_THREADS) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += Zraw[i * d + f];
    const double mu = s / (double)n;
    double v = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double t = Zraw[i * d + f] - mu;
      v = fma(t, t, v);
    }
    var[f] = v / (double)n;
  }
  __syncthreads();
  if (tid == 0) {
    // insertion sort of the d <= 256 variances
    for (int64_t i = 1; i < d; ++i) {
      const double x = var[i];
      int64_t j = i - 1;
      while (j >= 0 && var[j] > x) {
        var[j + 1] = var[j];
        --j;
      }
      var[j + 1] = x;
    }
    for (int k = 0; k < 8; ++k) res[k] = quantile_sorted(var, d, (double)k / 7.0);
  }
  // log Euclidean distances over all pairs i < j of the subsample
  const int64_t npairs = nsub * (nsub - 1) / 2;
  for (int64_t p = tid; p < len; p += ST_THREADS) {
    if (p < npairs) {
      // decode p -> (i, j), i < j, row-major over the strict upper triangle
      int64_t i = (int64_t)((2.0 * nsub - 1.0 - sqrt((2.0 * nsub - 1.0) * (2.0 * nsub - 1.0) - 8.0 * (double)p)) * 0.5);
      while (i > 0 && i * (2 * nsub - i - 1) / 2 > p) --i;
      while ((i + 1) * (2 * nsub - i - 2) / 2 <= p) ++i;
      const int64_t j = p - i * (2 * nsub - i - 1) / 2 + i + 1;
      const double* a = Zstd + sub[i] * d;
      const double* b = Zstd + sub[j] * d;
      double s = 0.0;
      for (int64_t f = 0; f < d; ++f) {
        const double t = a[f] - b[f];
        s = fma(t, t, s);
      }
      work[p] = 0.5 * log(s);
    } else {
      work[p] = INFINITY;
    }
  }
  __syncthreads();
  bitonic_sort(work, len);
  if (tid < 23) res[8 + tid] = quantile_sorted(work, npairs, (double)(tid + 1) / 24.0);
  // log population variance of the raw targets
  double s = 0.0;
  for (int64_t i = tid; i < n; i += ST_THREADS) s += yraw[i];
  red[tid] = s;
  __syncthreads();
  for (int w = ST_THREADS / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double mu = red[0] / (double)n;
  __syncthreads();
  double v = 0.0;
  for (int64_t i = tid; i < n; i += ST_THREADS) {
    const double t = yraw[i] - mu;
    v = fma(t, t, v);
  }
  red[tid] = v;
  __syncthreads();
  for (int w = ST_THREADS / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) res[31] = log(red[0] / (double)n);
  __syncthreads();
  if (tid < 32) {
    if (out64) out64[tid] = res[tid];
    if (out32) out32[tid] = (float)res[tid];
  }
}

int64_t stats_sort_len(int64_t nsub) {
  const int64_t np = nsub * (nsub - 1) / 2;
  int64_t len = 1;
  while (len < np) len <<= 1;
  return len;
}

hipError_t launch_summary_stats(const double* Zraw, const double* Zstd, const double* yraw, int64_t n, int64_t d,
                                const int64_t* sub, int64_t nsub, double* work, double* out64, float* out32,
                                hipStream_t st) {
  hipLaunchKernelGGL(summary_stats_kernel, dim3(1), dim3(ST_THREADS), 0, st, Zraw, Zstd, yraw, n, d, sub, nsub, work,
                     stats_sort_len(nsub), out64, out32);
  return hipGetLastError();
}

// ---------------------------------------------------------------- network
constexpr int MLP_IN = 32, MLP_H = 128, MLP_OUT = 3;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_OUT * MLP_H, MLP_NPARAM = OFF_B3 + MLP_OUT;
constexpr int MLP_THREADS = 1024;

GPR_DEV float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
GPR_DEV float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// act: [a1 | a2 | h1 | h2 | out | dout | d2 | d1], each B x 128 except out/dout (B x 3)
struct MlpArgs {
  float* params;
  float* m;
  float* v;
  float* grad;          // optional: gradient out (21,123)
  const float* X;       // B x 32
  const float* Y;       // B x 3 (training) or null (inference)
  float* out;           // B x 3 network output (optional)
  float* loss;          // optional scalar
  float* act;           // workspace
  int B;
  int mode;             // 0: forward only, 1: loss + gradient, 2: loss + gradient + Adam
  float lr, b1, b2, eps;
  int t;                // Adam step (1-based)
};

__global__ __launch_bounds__(MLP_THREADS)
void mlp_kernel(MlpArgs a) {
  __shared__ float red[MLP_THREADS];
  const int tid = threadIdx.x;
  const int B = a.B;
  const float* W1 = a.params + OFF_W1;
  const float* b1 = a.params + OFF_B1;
  const float* W2 = a.params + OFF_W2;
  const float* b2 = a.params + OFF_B2;
  const float* W3 = a.params + OFF_W3;
  const float* b3 = a.params + OFF_B3;
  float* a1 = a.act;
  float* a2 = a1 + (int64_t)B * MLP_H;
  float* h1 = a2 + (int64_t)B * MLP_H;
  float* h2 = h1 + (int64_t)B * MLP_H;
  float* out = h2 + (int64_t)B * MLP_H;
  float* dout = out + (int64_t)B * MLP_OUT;
  float* d2 = dout + (int64_t)B * MLP_OUT;
  float* d1 = d2 + (int64_t)B * MLP_H;
  // layer 1
  for (int e = tid; e < B * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, o = e % MLP_H;
    float s = b1[o];
    for (int i = 0; i < MLP_IN; ++i) s = fmaf(a.X[r * MLP_IN + i], W1[o * MLP_IN + i], s);
    a1[e] = s;
    h1[e] = gelu_f(s);
  }
  __syncthreads();
  // layer 2
  for (int e = tid; e < B * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, o = e % MLP_H;
    float s = b2[o];
    for (int i = 0; i < MLP_H; ++i) s = fmaf(h1[r * MLP_H + i], W2[o * MLP_H + i], s);
    a2[e] = s;
    h2[e] = gelu_f(s);
  }
  __syncthreads();
  // layer 3
  for (int e = tid; e < B * MLP_OUT; e += MLP_THREADS) {
    const int r = e / MLP_OUT, o = e % MLP_OUT;
    float s = b3[o];
    for (int i = 0; i < MLP_H; ++i) s = fmaf(h2[r * MLP_H + i], W3[o * MLP_H + i], s);
    out[e] = s;
    if (a.out) a.out[e] = s;
  }
  __syncthreads();
  if (a.mode == 0) return;
  // mean-squared error and its gradient at the output
  const float scale = 2.0f / (float)(B * MLP_OUT);
  float ls = 0.0f;
  for (int e = tid; e < B * MLP_OUT; e += MLP_THREADS) {
    const float df = out[e] - a.Y[e];
    dout[e] = scale * df;
    ls = fmaf(df, df, ls);
  }
  red[tid] = ls;
  __syncthreads();
  for (int w = MLP_THREADS / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && a.loss) a.loss[0] = red[0] / (float)(B * MLP_OUT);
  float* g = a.grad;
  // output layer: gW3, gb3 and d2 = (dout W3) o gelu'(a2)
  for (int e = tid; e < MLP_OUT * MLP_H + MLP_OUT; e += MLP_THREADS) {
    float s = 0.0f;
    if (e < MLP_OUT * MLP_H) {
      const int o = e / MLP_H, i = e % MLP_H;
      for (int r = 0; r < B; ++r) s = fmaf(dout[r * MLP_OUT + o], h2[r * MLP_H + i], s);
    } else {
      const int o = e - MLP_OUT * MLP_H;
      for (int r = 0; r < B; ++r) s += dout[r * MLP_OUT + o];
    }
    g[OFF_W3 + e] = s;
  }
  for (int e = tid; e < B * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, i = e % MLP_H;
    float s = 0.0f;
    for (int o = 0; o < MLP_OUT; ++o) s = fmaf(dout[r * MLP_OUT + o], W3[o * MLP_H + i], s);
    d2[e] = s * gelu_grad_f(a2[e]);
  }
  __syncthreads();
  // hidden layer 2: gW2, gb2 and d1 = (d2 W2) o gelu'(a1)
  for (int e = tid; e < MLP_H * MLP_H + MLP_H; e += MLP_THREADS) {
    float s = 0.0f;
    if (e < MLP_H * MLP_H) {
      const int o = e / MLP_H, i = e % MLP_H;
      for (int r = 0; r < B; ++r) s = fmaf(d2[r * MLP_H + o], h1[r * MLP_H + i], s);
    } else {
      const int o = e - MLP_H * MLP_H;
      for (int r = 0; r < B; ++r) s += d2[r * MLP_H + o];
    }
    g[OFF_W2 + e] = s;
  }
  for (int e = tid; e < B * MLP_H; e += MLP_THREADS) {
    const int r = e / MLP_H, i = e % MLP_H;
    float s = 0.0f;
    for (int o = 0; o < MLP_H; ++o) s = fmaf(d2[r * MLP_H + o], W2[o * MLP_H + i], s);
    d1[e] = s * gelu_grad_f(a1[e]);
  }
  __syncthreads();
  // input layer: gW1, gb1
  for (int e = tid; e < MLP_H * MLP_IN + MLP_H; e += MLP_THREADS) {
    float s = 0.0f;
    if (e < MLP_H * MLP_IN) {
      const int o = e / MLP_IN, i = e % MLP_IN;
      for (int r = 0; r < B; ++r) s = fmaf(d1[r * MLP_H + o], a.X[r * MLP_IN + i], s);
    } else {
      const int o = e - MLP_H * MLP_IN;
      for (int r = 0; r < B; ++r) s += d1[r * MLP_H + o];
    }
    g[OFF_W1 + e] = s;
  }
  __syncthreads();
  if (a.mode < 2) return;
  // Adam with bias correction
  const float c1 = 1.0f - powf(a.b1, (float)a.t), c2 = 1.0f - powf(a.b2, (float)a.t);
  for (int e = tid; e < MLP_NPARAM; e += MLP_THREADS) {
    const float gg = g[e];
    const float mm = a.b1 * a.m[e] + (1.0f - a.b1) * gg;
    const float vv = a.b2 * a.v[e] + (1.0f - a.b2) * gg * gg;
    a.m[e] = mm;
    a.v[e] = vv;
    a.params[e] -= a.lr * (mm / c1) / (sqrtf(vv / c2) + a.eps);
  }
}

int mlp_nparams() { return MLP_NPARAM; }

size_t mlp_act_floats(int B) { return (size_t)B * (6 * MLP_H + 2 * MLP_OUT); }

hipError_t launch_mlp(float* params, float* m, float* v, float* grad, const float* X, const float* Y, float* out,
                      float* loss, float* act, int B, int mode, float lr, float b1, float b2, float eps, int t,
                      hipStream_t st) {
  MlpArgs a{params, m, v, grad, X, Y, out, loss, act, B, mode, lr, b1, b2, eps, t};
  hipLaunchKernelGGL(mlp_kernel, dim3(1), dim3(MLP_THREADS), 0, st, a);
  return hipGetLastError();
}

}  // namespace gpr
