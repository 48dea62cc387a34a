// Generic travel-time network kernel (any H <= 256, any D): FP32 vector ALU,
// forward-mode source gradient.
//
// Alongside each activation a_l it carries the three tangents da_l/du_c of
// the source inputs (c = 0, 1, 2):  da_1/du_c = (1 - a_1^2) W_0[:, c],
// da_{l+1}/du_c = (1 - a_{l+1}^2) (W_l da_l/du_c), do/du_c = w_out . da_D/du_c.
// This is the same derivative as the paper's reverse-mode AD (Sec. 3.2) with
// no stored activations at all; it serves the FP32 path of shapes the
// matrix-core kernels do not instantiate.
//
// Block: 256 threads, TR rows.  Thread t owns neuron t % H for rows
// t / H, t / H + 256 / H, ...  LDS holds the current layer as
// [TR][H][4] floats (activation, three tangents) and the next one.
#include "internal.h"

namespace spider {

namespace {

constexpr int kTR = 8;

__global__ __launch_bounds__(256) void k_mlp_tangent(RowSource src, NetView net, RowOut* out) {
  extern __shared__ float4 lds4[];
  const int H = net.H;
  const int D = net.D;
  const int t = threadIdx.x;
  const int nrg = 256 / H;          // row groups
  const int n = t % H;
  const int rg = t / H;
  const bool active = rg < nrg;
  float4* cur = lds4;               // [kTR][H]
  float4* nxt = lds4 + kTR * H;
  __shared__ float u_s[kTR][6];
  const int64_t row0 = (int64_t)blockIdx.x * kTR;

  if (t < kTR) {
    const int64_t r = row0 + t;
    float u[6] = {0, 0, 0, 0, 0, 0};
    if (r < src.rows) row_inputs(src, net, r, u);
    for (int c = 0; c < 6; ++c) u_s[t][c] = u[c];
  }
  __syncthreads();

  // first layer, 6 -> H
  if (active) {
    const float* w0 = net.W0 + n * 6;
    const float b0 = net.bias[n];
    for (int r = rg; r < kTR; r += nrg) {
      float z = b0;
      for (int c = 0; c < 6; ++c) z += w0[c] * u_s[r][c];
      float a, d;
      tanh_d(z, a, d);
      cur[r * H + n] = make_float4(a, d * w0[0], d * w0[1], d * w0[2]);
    }
  }
  __syncthreads();

  // hidden layers
  for (int l = 1; l < D; ++l) {
    const float* wt = net.Wt + (int64_t)(l - 1) * H * H;
    const float bl = net.bias[l * H + n];
    float acc[kTR][4];
#pragma unroll
    for (int j = 0; j < kTR; ++j) acc[j][0] = acc[j][1] = acc[j][2] = acc[j][3] = 0.0f;
    if (active) {
      for (int k = 0; k < H; ++k) {
        const float w = wt[k * H + n];
#pragma unroll
        for (int j = 0; j < kTR; ++j) {
          const int r = rg + j * nrg;
          if (r < kTR) {
            const float4 v = cur[r * H + k];
            acc[j][0] += w * v.x;
            acc[j][1] += w * v.y;
            acc[j][2] += w * v.z;
            acc[j][3] += w * v.w;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kTR; ++j) {
        const int r = rg + j * nrg;
        if (r < kTR) {
          float a, d;
          tanh_d(acc[j][0] + bl, a, d);
          nxt[r * H + n] = make_float4(a, d * acc[j][1], d * acc[j][2], d * acc[j][3]);
        }
      }
    }
    __syncthreads();
    float4* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }

  // output layer: o = w_out . a_D + b_out, do/du_c = w_out . da_D/du_c
  __shared__ float fin[kTR][4];
  if (t < kTR * 4) {
    const int r = t / 4;
    const int comp = t % 4;
    float s = 0.0f;
    for (int k = 0; k < H; ++k) {
      const float4 v = cur[r * H + k];
      const float x = comp == 0 ? v.x : (comp == 1 ? v.y : (comp == 2 ? v.z : v.w));
      s += net.wout[k] * x;
    }
    fin[r][comp] = s;
  }
  __syncthreads();
  if (t < kTR) {
    const int64_t r = row0 + t;
    if (r < src.rows) {
      RowOut o;
      o.o = fin[t][0] + net.bout;
      o.d0 = fin[t][1];
      o.d1 = fin[t][2];
      o.d2 = fin[t][3];
      out[r] = o;
    }
  }
}

}  // namespace

hipError_t launch_mlp_tangent(const RowSource& src, const NetView& net, RowOut* out,
                              hipStream_t stream) {
  if (net.H < 1 || net.H > 256 || net.D < 1) return hipErrorNotSupported;
  if (src.rows == 0) return hipSuccess;
  const size_t lds = (size_t)2 * kTR * net.H * sizeof(float4);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_mlp_tangent,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kTR * 256 * 16);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int64_t blocks = ceil_div(src.rows, kTR);
  hipLaunchKernelGGL(k_mlp_tangent, dim3((unsigned)blocks), dim3(256), lds, stream, src, net, out);
  return hipGetLastError();
}

}  // namespace spider
