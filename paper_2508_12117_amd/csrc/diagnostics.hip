// Sampler diagnostics (Sec. 3.4 credibility intervals and calibration,
// Sec. 3.6 and Sec. 5 sampler health): over a device array of stored samples
// [S][P] (sample-major, P parameters per sample) -- percentiles, the rank of
// a reference value among the samples, the multi-chain effective sample
// size -- and the per-coordinate variance accumulation behind the ratio of
// stochastic-gradient variance to injected-noise variance.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace spider {
namespace {

constexpr int kQBlock = 256;
constexpr int kBlockD = 256;

inline unsigned grid_d(int64_t n) { return (unsigned)((n + kBlockD - 1) / kBlockD); }

// One workgroup per parameter: its S samples (stride P) are sorted in LDS by
// a bitonic network over the next power of two S2 (padded with +inf); the
// percentile of probability p is the linear interpolation between the order
// statistics around h = (S - 1) p.
__global__ void __launch_bounds__(kQBlock)
    k_quantiles(const double* samples, int64_t S, int64_t P, const double* probs, int n_probs,
                int S2, double* out) {
  extern __shared__ double v[];
  const int64_t p = blockIdx.x;
  for (int i = threadIdx.x; i < S2; i += kQBlock)
    v[i] = i < S ? samples[(int64_t)i * P + p] : INFINITY;
  __syncthreads();
  for (int k = 2; k <= S2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < S2; i += kQBlock) {
        const int l = i ^ j;
        if (l > i) {
          const bool ascending = (i & k) == 0;
          const double a = v[i], b = v[l];
          if ((a > b) == ascending) {
            v[i] = b;
            v[l] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int q = threadIdx.x; q < n_probs; q += kQBlock) {
    const double h = (double)(S - 1) * probs[q];
    const int64_t lo = (int64_t)floor(h);
    const int64_t hi = lo + 1 < S ? lo + 1 : lo;
    out[(int64_t)q * P + p] = v[lo] + (h - (double)lo) * (v[hi] - v[lo]);
  }
}

// frac[p] = (#{samples < value} + #{samples == value} / 2) / S.
__global__ void k_ranks(const double* samples, int64_t S, int64_t P, const double* values,
                        double* frac) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double x = values[p];
  int64_t below = 0, ties = 0;
  for (int64_t s = 0; s < S; ++s) {
    const double v = samples[s * P + p];
    below += v < x;
    ties += v == x;
  }
  frac[p] = ((double)below + 0.5 * (double)ties) / (double)S;
}

// Multi-chain effective sample size of each parameter over draws x[K][C][P]:
// chain means mu_c and variances s_c^2 (divisor K - 1), W = mean s_c^2,
// B/K = variance of the chain means (divisor C - 1, 0 for one chain),
// var+ = (K - 1)/K W + B/K; lag-t autocorrelation rho_t = 1 - (W - g_t)/var+
// with g_t the chains' mean of (1/K) sum_{i < K-t} (x_i - mu_c)(x_{i+t} - mu_c)
// and rho_0 = 1; pair sums P_k = rho_2k + rho_2k+1 are taken while positive
// and made non-increasing; tau = -1 + 2 sum P_k and ESS = C K / tau.
// var+ = 0 (constant draws) gives NaN.
__global__ void k_ess(const double* x, int64_t K, int C, int64_t P, double* ess) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double mu[kMaxEssChains];
  double W = 0.0, mbar = 0.0;
  for (int c = 0; c < C; ++c) {
    double s = 0.0;
    for (int64_t i = 0; i < K; ++i) s += x[(i * C + c) * P + p];
    mu[c] = s / (double)K;
    mbar += mu[c];
    double ss = 0.0;
    for (int64_t i = 0; i < K; ++i) {
      const double d = x[(i * C + c) * P + p] - mu[c];
      ss += d * d;
    }
    W += ss / (double)(K - 1);
  }
  W /= (double)C;
  mbar /= (double)C;
  double BK = 0.0;
  if (C > 1) {
    for (int c = 0; c < C; ++c) BK += (mu[c] - mbar) * (mu[c] - mbar);
    BK /= (double)(C - 1);
  }
  const double var_plus = (double)(K - 1) / (double)K * W + BK;
  if (!(var_plus > 0.0)) {
    ess[p] = NAN;
    return;
  }
  auto rho = [&](int64_t t) {
    if (t == 0) return 1.0;
    double g = 0.0;
    for (int c = 0; c < C; ++c) {
      double s = 0.0;
      for (int64_t i = 0; i + t < K; ++i)
        s += (x[(i * C + c) * P + p] - mu[c]) * (x[((i + t) * C + c) * P + p] - mu[c]);
      g += s / (double)K;
    }
    g /= (double)C;
    return 1.0 - (W - g) / var_plus;
  };
  double sum = 0.0, prev = INFINITY;
  for (int64_t k = 0; 2 * k + 1 < K; ++k) {
    double pk = rho(2 * k) + rho(2 * k + 1);
    if (!(pk > 0.0)) break;
    pk = fmin(pk, prev);
    prev = pk;
    sum += pk;
  }
  const double tau = -1.0 + 2.0 * sum;
  ess[p] = (double)C * (double)K / tau;
}

// Welford accumulation of the k-th (0-based) value of each coordinate.
__global__ void k_welford(const double* g, int64_t n, int64_t k, double* mean, double* m2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double x = g[q];
  const double mu = k == 0 ? 0.0 : mean[q];
  const double d = x - mu;
  const double nm = mu + d / (double)(k + 1);
  mean[q] = nm;
  m2[q] = (k == 0 ? 0.0 : m2[q]) + d * (x - nm);
}

// ratio = eps V Var(g) / (2 a^2), Var(g) = m2 / (K - 1), V = 1/(sqrt(v) + eps_p)
// (pSGLD) or 1; block partial sums of the ratios into part[block].
__global__ void k_noise_ratio(const double* m2, int64_t n, int64_t K, const double* v, int precond,
                              double eps_p, double step, double amp, double* ratio,
                              double* part) {
  __shared__ double sh[kBlockD];
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  if (q < n) {
    const double V = precond ? 1.0 / (sqrt(v[q]) + eps_p) : 1.0;
    r = step * V * (m2[q] / (double)(K - 1)) / (2.0 * amp * amp);
    ratio[q] = r;
  }
  sh[threadIdx.x] = r;
  __syncthreads();
  for (int w = kBlockD / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

}  // namespace

hipError_t launch_quantiles(const double* samples, int64_t S, int64_t P, const double* probs,
                            int n_probs, double* out, hipStream_t s) {
  int S2 = 1;
  while (S2 < S) S2 <<= 1;
  hipLaunchKernelGGL(k_quantiles, dim3((unsigned)P), dim3(kQBlock), (size_t)S2 * 8, s, samples, S,
                     P, probs, n_probs, S2, out);
  return hipGetLastError();
}

hipError_t launch_ranks(const double* samples, int64_t S, int64_t P, const double* values,
                        double* frac, hipStream_t s) {
  hipLaunchKernelGGL(k_ranks, dim3(grid_d(P)), dim3(kBlockD), 0, s, samples, S, P, values, frac);
  return hipGetLastError();
}

hipError_t launch_ess(const double* x, int64_t K, int C, int64_t P, double* ess, hipStream_t s) {
  hipLaunchKernelGGL(k_ess, dim3(grid_d(P)), dim3(kBlockD), 0, s, x, K, C, P, ess);
  return hipGetLastError();
}

void launch_welford(const double* g, int64_t n, int64_t k, double* mean, double* m2,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_welford, dim3(grid_d(n)), dim3(kBlockD), 0, s, g, n, k, mean, m2);
}

int64_t noise_ratio_blocks(int64_t n) { return grid_d(n); }

void launch_noise_ratio(const double* m2, int64_t n, int64_t K, const double* v, int precond,
                        double eps_p, double step, double amp, double* ratio, double* part,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_noise_ratio, dim3(grid_d(n)), dim3(kBlockD), 0, s, m2, n, K, v, precond,
                     eps_p, step, amp, ratio, part);
}

}  // namespace spider
