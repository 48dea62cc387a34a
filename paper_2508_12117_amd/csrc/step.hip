// Per-step kernels of the hot path that work per event (centroid, priors
// and the Langevin update, moments), the FP64 travel-time assembly of
// explicit rows, and the catalog preparation done once at load.  The
// minibatch pipeline itself (selection, CSR order, residuals, whitening,
// per-event reduction) is in batch_csr.hip.
//
//   centroid  per-chain mean of theta (fixed-order two-level reduction)
//   update    priors + SGLD / pSGLD (eq:pSGLD) + Philox noise + Welford
#include <climits>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "device_rng.h"
#include "internal.h"
#include "tt_assemble.h"

namespace spider {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = ceil_div(n, block);
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Fixed-order block sum of one double per thread (blockDim == TB).
template <int TB = kBlock>
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- load time

__global__ void k_pair_weights(const double* hypo0, const int2* pairs, int64_t P, double ell,
                               double p, double eps_w, double* w_pair) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const int2 ij = pairs[e];
  const double* a = hypo0 + (int64_t)ij.x * 4;
  const double* b = hypo0 + (int64_t)ij.y * 4;
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  const double d = sqrt(dx * dx + dy * dy + dz * dz);
  w_pair[e] = pow(d / ell, p) + eps_w;
}

// bad bits: 1 id out of range / i == j, 2 non-finite value, 4 source at a station
__global__ void k_validate(const double* hypo0, int M, const double* stations, int L,
                           const int2* pairs, int64_t P, const Obs* obs, int64_t N, int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int flag = 0;
  if (t < P) {
    const int2 ij = pairs[t];
    if (ij.x < 0 || ij.x >= M || ij.y < 0 || ij.y >= M || ij.x == ij.y) flag |= 1;
  }
  if (t < M) {
    for (int a = 0; a < 4; ++a)
      if (!isfinite(hypo0[t * 4 + a])) flag |= 2;
  }
  if (t < L) {
    for (int a = 0; a < 3; ++a)
      if (!isfinite(stations[t * 3 + a])) flag |= 2;
  }
  if (t < N) {
    const Obs o = obs[t];
    if (o.pair < 0 || o.pair >= P || o.sta < 0 || o.sta >= L) {
      flag |= 1;
    } else {
      if (!isfinite(o.dt)) flag |= 2;
      const int2 ij = pairs[o.pair];
      if (ij.x >= 0 && ij.x < M && ij.y >= 0 && ij.y < M) {
        const double* s = stations + (int64_t)o.sta * 3;
        for (int side = 0; side < 2; ++side) {
          const double* x = hypo0 + (int64_t)(side ? ij.y : ij.x) * 4;
          const double d2 = (x[0] - s[0]) * (x[0] - s[0]) + (x[1] - s[1]) * (x[1] - s[1]) +
                            (x[2] - s[2]) * (x[2] - s[2]);
          if (!(d2 >= 1e-6)) flag |= 4;
        }
      }
    }
  }
  if (flag) atomicOr(bad, flag);
}

__global__ void k_obs_group_keys(const Obs* obs, int64_t N, uint32_t* keys, uint32_t* vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  keys[t] = (uint32_t)obs[t].sta;
  vals[t] = (uint32_t)t;
}

// One block per group: binary search of the group's range in the sorted keys,
// then a fixed-order sum of its weights.
__global__ void k_group_mean(const uint32_t* keys, const uint32_t* vals, int64_t N, const Obs* obs,
                             const double* w_pair, double* inv_mean) {
  __shared__ double sh[kBlock];
  const uint32_t g = blockIdx.x;
  int64_t lo = 0, hi = N;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (keys[mid] < g) lo = mid + 1; else hi = mid;
  }
  const int64_t begin = lo;
  hi = N;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (keys[mid] <= g) lo = mid + 1; else hi = mid;
  }
  const int64_t end = lo;
  double s = 0.0;
  for (int64_t q = begin + threadIdx.x; q < end; q += kBlock) s += w_pair[obs[vals[q]].pair];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) inv_mean[g] = end > begin ? (double)(end - begin) / s : 0.0;
}

__global__ void k_mean4(const double* a, int64_t rows, double* out) {
  __shared__ double sh[kBlock];
  for (int c = 0; c < 4; ++c) {
    double s = 0.0;
    for (int64_t m = threadIdx.x; m < rows; m += kBlock) s += a[m * 4 + c];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = s / (double)rows;
  }
}

// ---------------------------------------------------------------- step

__global__ void k_pack_obs(const Obs* obs, int64_t N, const int2* pairs, const double* w_pair,
                           const double* inv_mean, ObsRec* rec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const Obs ob = obs[t];
  const int2 ij = pairs[ob.pair];
  ObsRec r;
  r.i = ij.x;
  r.j = ij.y;
  r.g = ob.sta;
  r.dt = ob.dt;
  r.w = w_pair[ob.pair] * inv_mean[ob.sta];
  r.pad = 0.0;
  rec[t] = r;
}

// ---- centroid, update, gradient assembly

constexpr int kCentroidChunk = 4096;

__global__ void k_centroid_partial(const double* theta, int M, int nchunk, double* partial) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.y;
  const int chunk = blockIdx.x;
  const double* th = theta + (int64_t)c * M * 4;
  const int64_t m0 = (int64_t)chunk * kCentroidChunk;
  const int64_t m1 = min((int64_t)M, m0 + kCentroidChunk);
  // one pass over the chunk's events, each read as one 32-byte load
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t m = m0 + threadIdx.x; m < m1; m += kBlock) {
    const double4 x = *(const double4*)(th + m * 4);
    s[0] += x.x;
    s[1] += x.y;
    s[2] += x.z;
    s[3] += x.w;
  }
  for (int a = 0; a < 4; ++a) {
    const double t = block_sum(s[a], sh);
    if (threadIdx.x == 0) partial[((int64_t)c * nchunk + chunk) * 4 + a] = t;
  }
}

__global__ void k_centroid_final(const double* partial, int nchunk, int M, double* thetabar) {
  const int c = blockIdx.x;
  const int a = threadIdx.x;
  if (a >= 4) return;
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += partial[((int64_t)c * nchunk + k) * 4 + a];
  thetabar[c * 4 + a] = s / (double)M;
}

struct UpdateKArgs {
  double step, beta2, eps_p, noise_scale;
  int precond;
  uint32_t k0, k1;
  int64_t burn, thin;
  double* samples;
  int64_t sample_cap;
  int sample_C;
};

__device__ inline bool records(int64_t t, int64_t burn, int64_t thin) {
  return t >= burn && (t - burn) % thin == 0;
}

__global__ void k_update(CatView cat, int C, double* theta, double* v, const double* G,
                         const double* thetabar, const int64_t* steps, const int64_t* mcount,
                         UpdateKArgs a, double* mean, double* m2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)C * cat.M) return;
  const int c = (int)(q / cat.M);
  const int64_t m = q - (int64_t)c * cat.M;
  const int64_t t = steps[c];
  double eta[4];
  noise4(a.k0, a.k1, cat.stream, (uint32_t)c, (uint32_t)t, (uint32_t)m, eta);
  double x[4];
  for (int k = 0; k < 4; ++k) {
    const double th = theta[q * 4 + k];
    const double sp = cat.prior_sigma[k], sc = cat.centroid_sigma[k];
    const double g = G[q * 4 + k] - (th - cat.hypo0[m * 4 + k]) / (sp * sp) -
                     (thetabar[c * 4 + k] - cat.mu_c[k]) / (sc * sc) / (double)cat.M;
    double nt;
    if (a.precond == 0) {
      nt = th + a.step * g + a.noise_scale * sqrt(2.0 * a.step) * eta[k];
    } else {
      const double vv = a.beta2 * v[q * 4 + k] + (1.0 - a.beta2) * g * g;
      v[q * 4 + k] = vv;
      const double V = 1.0 / (sqrt(vv) + a.eps_p);
      nt = th + a.step * V * g + a.noise_scale * sqrt(2.0 * a.step * V) * eta[k];
    }
    theta[q * 4 + k] = nt;
    x[k] = nt;
  }
  if (records(t, a.burn, a.thin)) {
    const double cnt = (double)(mcount[c] + 1);
    double d[4], after[4];
    for (int k = 0; k < 4; ++k) {
      const double mu = mean[q * 4 + k];
      d[k] = x[k] - mu;
      const double nm = mu + d[k] / cnt;
      mean[q * 4 + k] = nm;
      after[k] = x[k] - nm;
    }
    int u = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j, ++u) m2[q * 10 + u] += d[i] * after[j];
    const int64_t slot = mcount[c];
    if (a.samples && slot < a.sample_cap) {
      double* o = a.samples + ((slot * a.sample_C + c) * (int64_t)cat.M + m) * 4;
      for (int k = 0; k < 4; ++k) o[k] = x[k];
    }
  }
}

// Adam on the loss whose negative gradient is G (Stage 1, Sec. 3.2): with
// g = -G, m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, and k = the chain's
// step counter + 1, theta -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
__global__ void k_adam(int C, int M, double* theta, double* m, double* v, const double* G,
                       const int64_t* steps, AdamArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)C * M * 4) return;
  const int c = (int)(q / ((int64_t)M * 4));
  const double k = (double)(steps[c] + 1);
  const double g = -G[q];
  const double mq = a.beta1 * m[q] + (1.0 - a.beta1) * g;
  const double vq = a.beta2 * v[q] + (1.0 - a.beta2) * g * g;
  m[q] = mq;
  v[q] = vq;
  const double mh = mq / (1.0 - pow(a.beta1, k));
  const double vh = vq / (1.0 - pow(a.beta2, k));
  theta[q] -= a.lr * mh / (sqrt(vh) + a.eps);
}

__global__ void k_advance(int C, int64_t* steps, int64_t* mcount, int64_t burn, int64_t thin) {
  const int c = threadIdx.x + blockIdx.x * blockDim.x;
  if (c >= C) return;
  if (records(steps[c], burn, thin)) mcount[c] += 1;
  steps[c] += 1;
}

__global__ void k_grad_finish(CatView cat, const double* theta, const double* G,
                              const double* thetabar, unsigned flags, double* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)cat.M * 4) return;
  const int k = (int)(q & 3);
  double g = G[q];
  if (flags & 1u) {
    const double sp = cat.prior_sigma[k];
    g -= (theta[q] - cat.hypo0[q]) / (sp * sp);
  }
  if (flags & 2u) {
    const double sc = cat.centroid_sigma[k];
    g -= (thetabar[k] - cat.mu_c[k]) / (sc * sc) / (double)cat.M;
  }
  out[q] = g;
}

// partial sums of -scale/2 r z (blocks of the batch) and the event prior
__global__ void k_logpost_partial(CatView cat, int64_t n, double scale, const double* r,
                                  const double* z, const double* theta, unsigned flags,
                                  double* tmp) {
  __shared__ double sh[kBlock];
  const int64_t per = ceil_div(n, (int64_t)gridDim.x);
  const int64_t q0 = (int64_t)blockIdx.x * per, q1 = min(n, q0 + per);
  double s = 0.0;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) s += r[q] * z[q];
  s = -0.5 * scale * block_sum(s, sh);
  double pr = 0.0;
  if (flags & 1u) {
    const int64_t per_m = ceil_div((int64_t)cat.M * 4, (int64_t)gridDim.x);
    const int64_t m0 = (int64_t)blockIdx.x * per_m, m1 = min((int64_t)cat.M * 4, m0 + per_m);
    for (int64_t q = m0 + threadIdx.x; q < m1; q += kBlock) {
      const double d = (theta[q] - cat.hypo0[q]) / cat.prior_sigma[q & 3];
      pr += d * d;
    }
    pr = -0.5 * block_sum(pr, sh);
  }
  if (threadIdx.x == 0) tmp[blockIdx.x] = s + pr;
}

__global__ void k_logpost_final(CatView cat, const double* tmp, int nb, const double* thetabar,
                                unsigned flags, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nb; ++k) s += tmp[k];
  if (flags & 2u) {
    for (int k = 0; k < 4; ++k) {
      const double d = (thetabar[k] - cat.mu_c[k]) / cat.centroid_sigma[k];
      s += -0.5 * d * d;
    }
  }
  *out = s;
}

// T and dT/dx of explicit rows from the network outputs; with vjp_w the
// source gradient is written scaled by the row's weight, w dT/dx (the
// vector-Jacobian product of a reverse sweep through T).  T may be null.
__global__ void k_tt_assemble(NetView net, int64_t rows, const double* x, const double* s,
                              const RowOut* out, double* T, double* gradT, const double* vjp_w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double xx[3] = {x[r * 3], x[r * 3 + 1], x[r * 3 + 2]};
  const double ss[3] = {s[r * 3], s[r * 3 + 1], s[r * 3 + 2]};
  double tt, g[3];
  assemble_tt(net, xx, ss, out[r], tt, g);
  if (T) T[r] = tt;
  if (gradT) {
    const double w = vjp_w ? vjp_w[r] : 1.0;
    gradT[r * 3] = w * g[0];
    gradT[r * 3 + 1] = w * g[1];
    gradT[r * 3 + 2] = w * g[2];
  }
}

__global__ void k_noise(CatView cat, uint32_t k0, uint32_t k1, int chain, uint32_t step,
                        double* eta) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= cat.M) return;
  double e[4];
  noise4(k0, k1, cat.stream, (uint32_t)chain, step, (uint32_t)m, e);
  for (int k = 0; k < 4; ++k) eta[m * 4 + k] = e[k];
}

__global__ void k_finite(const double* a, int64_t count, int64_t per_chain, int* bad_chain) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  if (!isfinite(a[q])) atomicMin(bad_chain, (int)(q / per_chain));
}

__global__ void k_pool_moments(int C, int M, const double* mean, const double* m2,
                               const int64_t* cnt, double* out_mean, double* out_cov) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double mu[4] = {0, 0, 0, 0}, s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double n = 0.0;
  for (int c = 0; c < C; ++c) {
    const double nc = (double)cnt[c];
    if (nc == 0.0) continue;
    const double* mc = mean + ((int64_t)c * M + m) * 4;
    const double* sc = m2 + ((int64_t)c * M + m) * 10;
    const double nn = n + nc;
    double d[4];
    for (int k = 0; k < 4; ++k) d[k] = mc[k] - mu[k];
    const double f = n * nc / nn;
    int u = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j, ++u) s[u] += sc[u] + d[i] * d[j] * f;
    for (int k = 0; k < 4; ++k) mu[k] += d[k] * (nc / nn);
    n = nn;
  }
  if (out_mean)
    for (int k = 0; k < 4; ++k) out_mean[m * 4 + k] = mu[k];
  if (out_cov) {
    const double div = n > 1.0 ? n - 1.0 : 1.0;
    for (int u = 0; u < 10; ++u) out_cov[m * 10 + u] = s[u] / div;
  }
}

__global__ void k_fill(double* p, double v, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

// ---- outlier screening after Stage 1

__global__ void k_iota(int64_t* idx, int64_t start, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) idx[t] = start + t;
}

__global__ void k_absdev(const double* r, int64_t N, double med, double* d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) d[t] = fabs(r[t] - med);
}

// Adds the block's sum of k (one value per thread) to *count.
__device__ void block_count_add(unsigned int k, unsigned long long* count) {
  __shared__ unsigned int sh[kBlock];
  sh[threadIdx.x] = k;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0]) atomicAdd(count, (unsigned long long)sh[0]);
}

// keep[i] = |r_i - med| <= thr; the kept count is added to *count.
__global__ void k_keep(const double* r, int64_t N, double med, double thr, uint8_t* keep,
                       unsigned long long* count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned int k = 0;
  if (t < N) {
    k = fabs(r[t] - med) <= thr ? 1u : 0u;
    keep[t] = (uint8_t)k;
  }
  block_count_add(k, count);
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_pack_obs(const Obs* obs, int64_t N, const int2* pairs, const double* w_pair,
                     const double* inv_mean, ObsRec* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_obs, dim3(grid_for(N)), dim3(kBlock), 0, s, obs, N, pairs, w_pair,
                     inv_mean, rec);
}

void launch_pair_weights(const double* hypo0, const int2* pairs, int64_t P, double ell, double p,
                         double eps_w, double* w_pair, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_weights, dim3(grid_for(P)), dim3(kBlock), 0, s, hypo0, pairs, P, ell,
                     p, eps_w, w_pair);
}

void launch_validate(const double* hypo0, int M, const double* stations, int L, const int2* pairs,
                     int64_t P, const Obs* obs, int64_t N, int* bad, hipStream_t s) {
  int64_t mx = N;
  if (P > mx) mx = P;
  if (M > mx) mx = M;
  if (L > mx) mx = L;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(mx)), dim3(kBlock), 0, s, hypo0, M, stations, L,
                     pairs, P, obs, N, bad);
}

hipError_t group_inverse_mean(const Obs* obs, int64_t N, int L, const double* w_pair,
                              double* inv_mean, hipStream_t s) {
  uint32_t *k0 = nullptr, *k1 = nullptr, *v0 = nullptr, *v1 = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  hipError_t e = hipSuccess;
  int end_bit = 1;
  while ((1 << end_bit) < L) ++end_bit;
  do {
    if ((e = hipMallocAsync((void**)&k0, N * 4, s)) != hipSuccess) break;
    if ((e = hipMallocAsync((void**)&k1, N * 4, s)) != hipSuccess) break;
    if ((e = hipMallocAsync((void**)&v0, N * 4, s)) != hipSuccess) break;
    if ((e = hipMallocAsync((void**)&v1, N * 4, s)) != hipSuccess) break;
    hipLaunchKernelGGL(k_obs_group_keys, dim3(grid_for(N)), dim3(kBlock), 0, s, obs, N, k0, v0);
    if ((e = rocprim::radix_sort_pairs(nullptr, temp_bytes, k0, k1, v0, v1, (size_t)N, 0, end_bit,
                                       s)) != hipSuccess)
      break;
    if ((e = hipMallocAsync(&temp, temp_bytes, s)) != hipSuccess) break;
    if ((e = rocprim::radix_sort_pairs(temp, temp_bytes, k0, k1, v0, v1, (size_t)N, 0, end_bit,
                                       s)) != hipSuccess)
      break;
    hipLaunchKernelGGL(k_group_mean, dim3(L), dim3(kBlock), 0, s, k1, v1, N, obs, w_pair,
                       inv_mean);
    e = hipGetLastError();
  } while (false);
  (void)hipFreeAsync(k0, s);
  (void)hipFreeAsync(k1, s);
  (void)hipFreeAsync(v0, s);
  (void)hipFreeAsync(v1, s);
  if (temp) (void)hipFreeAsync(temp, s);
  return e;
}

void launch_mean4(const double* a, int64_t rows, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mean4, dim3(1), dim3(kBlock), 0, s, a, rows, out);
}

void launch_centroid(const double* theta, int C, int M, double* partial, double* thetabar,
                     hipStream_t s) {
  const int nchunk = (int)ceil_div(M, kCentroidChunk);
  hipLaunchKernelGGL(k_centroid_partial, dim3(nchunk, C), dim3(kBlock), 0, s, theta, M, nchunk,
                     partial);
  hipLaunchKernelGGL(k_centroid_final, dim3(C), dim3(64), 0, s, partial, nchunk, M, thetabar);
}

void launch_advance(int C, int64_t* steps, int64_t* mcount, const UpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(grid_for(C, 64)), dim3(64), 0, s, C, steps, mcount, a.burn,
                     a.thin);
}

void launch_update(const CatView& cat, int C, double* theta, double* v, const double* G,
                   const double* thetabar, int64_t* steps, int64_t* mcount, const UpdateArgs& a,
                   double* mean, double* m2, hipStream_t s, bool advance) {
  UpdateKArgs k;
  k.step = a.step;
  k.beta2 = a.beta2;
  k.eps_p = a.eps_p;
  k.noise_scale = a.noise_scale;
  k.precond = a.precond;
  k.k0 = (uint32_t)a.seed;
  k.k1 = (uint32_t)(a.seed >> 32);
  k.burn = a.burn;
  k.thin = a.thin;
  k.samples = a.samples;
  k.sample_cap = a.sample_cap;
  k.sample_C = a.sample_C;
  hipLaunchKernelGGL(k_update, dim3(grid_for((int64_t)C * cat.M)), dim3(kBlock), 0, s, cat, C,
                     theta, v, G, thetabar, steps, mcount, k, mean, m2);
  if (advance) launch_advance(C, steps, mcount, a, s);
}

void launch_adam(int C, int M, double* theta, double* m, double* v, const double* G,
                 int64_t* steps, const AdamArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for((int64_t)C * M * 4)), dim3(kBlock), 0, s, C, M, theta,
                     m, v, G, steps, a);
  // the step counters advance; no step of this stage records moments
  hipLaunchKernelGGL(k_advance, dim3(grid_for(C, 64)), dim3(64), 0, s, C, steps, (int64_t*)nullptr,
                     INT64_MAX, (int64_t)1);
}

void launch_grad_finish(const CatView& cat, const double* theta, const double* G,
                        const double* thetabar, unsigned flags, double* grad_out, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_finish, dim3(grid_for((int64_t)cat.M * 4)), dim3(kBlock), 0, s, cat,
                     theta, G, thetabar, flags, grad_out);
}

void launch_logpost(const CatView& cat, int64_t n, double scale, const double* r, const double* z,
                    const double* theta, const double* thetabar, unsigned flags, double* tmp,
                    double* out, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(k_logpost_partial, dim3(nb), dim3(kBlock), 0, s, cat, n, scale, r, z, theta,
                     flags, tmp);
  hipLaunchKernelGGL(k_logpost_final, dim3(1), dim3(64), 0, s, cat, tmp, nb, thetabar, flags, out);
}

void launch_tt_assemble(const NetView& net, int64_t rows, const double* x, const double* s,
                        const RowOut* out, double* T, double* gradT, const double* vjp_w,
                        hipStream_t st) {
  if (rows == 0) return;
  hipLaunchKernelGGL(k_tt_assemble, dim3(grid_for(rows)), dim3(kBlock), 0, st, net, rows, x, s,
                     out, T, gradT, vjp_w);
}

void launch_noise(const CatView& cat, uint64_t seed, int chain, int64_t step, double* eta,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_noise, dim3(grid_for(cat.M)), dim3(kBlock), 0, s, cat, (uint32_t)seed,
                     (uint32_t)(seed >> 32), chain, (uint32_t)step, eta);
}

void launch_finite(const double* a, int64_t count, int64_t per_chain, int* bad_chain,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_finite, dim3(grid_for(count)), dim3(kBlock), 0, s, a, count, per_chain,
                     bad_chain);
}

void launch_pool_moments(int C, int M, const double* mean, const double* m2, const int64_t* cnt,
                         double* out_mean, double* out_cov, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_moments, dim3(grid_for(M)), dim3(kBlock), 0, s, C, M, mean, m2, cnt,
                     out_mean, out_cov);
}

void launch_iota(int64_t* idx, int64_t start, int64_t len, hipStream_t s) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(len)), dim3(kBlock), 0, s, idx, start, len);
}

void launch_absdev(const double* r, int64_t N, double med, double* d, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_absdev, dim3(grid_for(N)), dim3(kBlock), 0, s, r, N, med, d);
}

void launch_keep(const double* r, int64_t N, double med, double thr, uint8_t* keep,
                 unsigned long long* count, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_keep, dim3(grid_for(N)), dim3(kBlock), 0, s, r, N, med, thr, keep, count);
}

hipError_t sort_doubles(const double* in, double* out, int64_t N, void* temp, size_t* temp_bytes,
                        hipStream_t s) {
  return rocprim::radix_sort_keys(temp, *temp_bytes, in, out, (size_t)N, 0, 64, s);
}

void launch_fill(double* p, double v, int64_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
}

}  // namespace spider
