// What the travel-time network kernels read: where their input rows come
// from, the network's device view, the per-row result, and the activation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spider {

// Where the network's input rows come from.
//  mode 0 (minibatch): row r is event ev[r] of chain r / rows_per_chain at
//          station sta[r]; x = theta[chain][ev][0:3], s = stations[sta].
//  mode 1 (explicit):  x = x[r][0:3], s = s[r][0:3].
//  mode 2 (several catalogs in one launch): rows [sub_row0[k], sub_row0[k+1])
//          are the rows of the mode-0 source sub[k] (device table, nsub
//          entries, sub_row0[nsub] = rows).
//  mode 3 (listed rows): row r is row list[r] of the mode-0 source.
struct RowSource {
  int mode;
  int nsub;
  const RowSource* sub;
  const int64_t* sub_row0;
  int64_t rows;
  const int32_t* ev;
  const int32_t* sta;
  const double* theta;
  int64_t rows_per_chain;
  int64_t theta_chain_stride;  // doubles between chains' states (M * 4)
  const double* stations;
  const double* x;
  const double* s;
  const int32_t* list;  // mode 3: row r of the launch is catalog row list[r]
};

// Network as the kernels see it (device pointers).
struct NetView {
  int D, H;
  const float* W0;     // [H][6]
  const float* bias;   // [D][H]: b[0] .. b[D-1]
  const float* W0s;    // kTanhScale * W0 (matrix-core kernels)
  const float* bias_s; // kTanhScale * bias
  const float* Wt;     // [D-1][H][H]: Wt[l][k][n] = W[l+1][n][k] (input-major)
  const float* wout;   // [H]
  float bout;
  double v0;
  double inv_v0;       // 1 / v0, rounded once on the host
  double center[3];
  double half[3];
  double inv_half[3];  // 1 / half, rounded once on the host
  const void* pack_fwd;  // matrix-core operand packs (precision dependent)
  const void* pack_bwd;
};

// Per-row network result: o and do/du for the three source inputs.
struct RowOut {
  float o, d0, d1, d2;
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Computes the network inputs u of row r.
__device__ inline void row_inputs(const RowSource& src_in, const NetView& net, int64_t r, float u[6]) {
  double x[3], s[3];
  const RowSource* sp = &src_in;
  if (src_in.mode == 2) {  // the catalog whose rows hold r: the last k with sub_row0[k] <= r
    int lo = 0, hi = src_in.nsub - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (src_in.sub_row0[mid] <= r) lo = mid;
      else hi = mid - 1;
    }
    r -= src_in.sub_row0[lo];
    sp = src_in.sub + lo;
  }
  const RowSource& src = *sp;
  if (src.mode == 0 || src.mode == 3) {
    if (src.mode == 3) r = src.list[r];
    const int64_t c = r / src.rows_per_chain;
    const double* th = src.theta + c * src.theta_chain_stride + (int64_t)src.ev[r] * 4;
    const double* st = src.stations + (int64_t)src.sta[r] * 3;
    const double4 e = *(const double4*)th;
    x[0] = e.x;
    x[1] = e.y;
    x[2] = e.z;
    for (int a = 0; a < 3; ++a) s[a] = st[a];
  } else {
    for (int a = 0; a < 3; ++a) {
      x[a] = src.x[r * 3 + a];
      s[a] = src.s[r * 3 + a];
    }
  }
  for (int a = 0; a < 3; ++a) {
    u[a] = (float)((x[a] - net.center[a]) * net.inv_half[a]);
    u[3 + a] = (float)((s[a] - net.center[a]) * net.inv_half[a]);
  }
}

// 2 log2(e): the matrix-core kernels carry it in their forward weights and
// biases, so that exp(2z) = 2^(kTanhScale z) is one hardware exponential.
constexpr double kTanhScale = 2.8853900817779268;

// tanh(z) and 1 - tanh(z)^2 from one exponential and one reciprocal: with
// e = exp(2|z|) and r = 1/(1 + e), tanh|z| = 1 - 2r and 1 - tanh^2 = 4r(1 - r),
// accurate also where tanh -> +-1 (e = inf gives r = 0).  exp uses the
// hardware base-2 exponential on 2 log2(e) |z|.
__device__ inline void tanh_d(float z, float& a, float& d) {
  const float e = __builtin_amdgcn_exp2f(fabsf(z) * 2.8853900817779268f);
  const float r = __builtin_amdgcn_rcpf(1.0f + e);
  a = copysignf(fmaf(r, -2.0f, 1.0f), z);
  d = 4.0f * r * (1.0f - r);
}

}  // namespace spider
