// Matrix-core travel-time network kernel for gfx950: forward pass and
// reverse-mode source gradient (Sec. 3.2) in one launch, BF16 operands with
// FP32 accumulation (v_mfma_f32_16x16x32_bf16) or FP32 throughout
// (v_mfma_f32_16x16x4_f32).
//
// Work split.  A workgroup of NW waves handles R = 16 RT rows.  Wave w owns
// the output neurons [16 CT w, 16 CT (w + 1)) of every hidden layer, in the
// forward pass and in the backward pass alike:
//   forward   z_{l+1}[:, own] = a_l[R, H] . W_l[own, H]^T      (A from LDS)
//   backward  e_l[:, own]     = e_{l+1}[R, H] . W_l[H, own]    (A from LDS)
// so the derivative factors d_l = 1 - a_l^2 that the backward pass needs at
// its own neurons were produced by the same lanes, in the same accumulator
// layout, and stay in registers between the passes: activations are never
// written to memory and nothing is recomputed.  Hidden-layer weights stream
// from L2 as pre-packed B operands: one 16-byte coalesced load per lane per
// chunk.  The 6-input first layer and the 1-output last layer are FP32 vector
// arithmetic on the accumulator layout.
//
// MFMA 16x16xK layouts used (lane l, c = l % 16, g = l / 16):
//   A: row c,  k-slots of group g      B: column c, k-slots of group g
//   C: column c, rows 4 g .. 4 g + 3
// The k index of slot (g, s, j) is g H/4 + s KPL + j for both operands; any
// such consistent assignment gives the full dot product.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace spider {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct PolBF16 {
  using T = __bf16;
  using V = bf16x8;                 // one MFMA operand per lane
  static constexpr int KPL = 8;     // k values per lane per MFMA
  static constexpr int RT = 4;      // row tiles per workgroup
  static constexpr bool kBF16 = true;
  __device__ static floatx4 mma(const V& a, const V& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

struct PolF32 {
  using T = float;
  using V = float;
  static constexpr int KPL = 1;
  static constexpr int RT = 2;
  static constexpr bool kBF16 = false;
  __device__ static floatx4 mma(const V& a, const V& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <class P>
struct Chunk {
  // 16 bytes of operand data per lane: SPC MFMA k-steps
  static constexpr int ELEMS = 16 / sizeof(typename P::T);
  static constexpr int SPC = ELEMS / P::KPL;
};

// Packed layout of one hidden layer (forward and backward alike):
// [col tile ct][chunk q][lane][ELEMS], column tile over the layer's outputs.
template <class P>
constexpr int chunks_per_layer(int H) {
  return (H / 4) / Chunk<P>::ELEMS;
}

template <class P, int H, int D, int NW>
struct Shape {
  static constexpr int CT = H / 16 / NW;       // column tiles per wave
  static constexpr int RT = P::RT;
  static constexpr int R = 16 * RT;            // rows per workgroup
  static constexpr int KG = H / 4;             // k per lane group
  static constexpr int NQ = chunks_per_layer<P>(H);
  static constexpr int PAD = 16 / sizeof(typename P::T);
  static constexpr int LDW = H + PAD;          // LDS row stride (elements)
  static constexpr int NL = D > 1 ? D - 1 : 1;  // stored derivative layers
  // derivative layers kept in registers; the rest go to LDS (BF16 pairs)
  static constexpr int NLR = (P::kBF16 && H * RT / NW > 64) ? (NL < 4 ? NL : 4) : NL;
  static constexpr int NLDS = NL - NLR;
  static constexpr int NT = NW * 64;
  static constexpr size_t ACT_BYTES = (size_t)R * LDW * sizeof(typename P::T);
  static constexpr size_t DLDS_BYTES = (size_t)NLDS * RT * CT * 2 * NT * 4;
  static constexpr size_t FIXED_BYTES = (size_t)R * 6 * 4 + (size_t)NW * R * 4 * 4;
  // two activation buffers when they fit in 160 KB of LDS, else one buffer
  // and an extra barrier per layer
  static constexpr int NBUF = 2 * ACT_BYTES + DLDS_BYTES + FIXED_BYTES <= 156 * 1024 ? 2 : 1;
  static_assert(NBUF * ACT_BYTES + DLDS_BYTES + FIXED_BYTES <= 160 * 1024, "LDS budget");
  static_assert(CT * NW * 16 == H, "H must split into 16-wide tiles over the waves");
  static_assert(NQ * Chunk<P>::ELEMS == KG, "H/4 must be a whole number of chunks");
};

// Derivative factors 1 - a^2 kept between the passes: FP32 registers, or in
// the BF16 path BF16 pairs (round to nearest even), the first NLR layers in
// registers and the rest in LDS, where each lane reads back only what it
// wrote ([layer][pair][thread] uint32, conflict-free).
template <class P, int NL, int NLR, int RT, int CT, int NT>
struct DStore {
  float v[NL][RT][CT][4];
  __device__ void set(int l, int rt, int ct, int i, float x) { v[l][rt][ct][i] = x; }
  __device__ float get(int l, int rt, int ct, int i) const { return v[l][rt][ct][i]; }
};

template <int NL, int NLR, int RT, int CT, int NT>
struct DStore<PolBF16, NL, NLR, RT, CT, NT> {
  uint32_t v[NLR][RT][CT][2];
  uint32_t* lds;  // [NL - NLR][RT * CT * 2][NT]
  int tid;
  uint32_t lo;
  __device__ void set(int l, int rt, int ct, int i, float x) {
    const uint32_t b = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
    if ((i & 1) == 0) {
      lo = b;
      return;
    }
    const uint32_t w = lo | (b << 16);
    if (l < NLR) v[l][rt][ct][i >> 1] = w;
    else lds[(((l - NLR) * RT * CT + rt * CT + ct) * 2 + (i >> 1)) * NT + tid] = w;
  }
  __device__ float get(int l, int rt, int ct, int i) const {
    const uint32_t w = l < NLR ? v[l][rt][ct][i >> 1]
                               : lds[(((l - NLR) * RT * CT + rt * CT + ct) * 2 + (i >> 1)) * NT + tid];
    return __uint_as_float((i & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
};

union Pack16 {
  uint4 u;
  bf16x8 b;
  float f[4];
};

template <class P, int H, int D, int NW>
__global__ __launch_bounds__(NW * 64) void k_mlp(RowSource src, NetView net, RowOut* out) {
  using S = Shape<P, H, D, NW>;
  using T = typename P::T;
  constexpr int CT = S::CT, RT = S::RT, R = S::R, NQ = S::NQ, LDW = S::LDW, KG = S::KG;
  constexpr int ELEMS = Chunk<P>::ELEMS, SPC = Chunk<P>::SPC;
  constexpr int NL = S::NL, NLR = S::NLR, NT = S::NT, NBUF = S::NBUF;

  __shared__ __attribute__((aligned(16))) T act[NBUF][R * LDW];
  __shared__ uint32_t dlds[S::NLDS > 0 ? S::NLDS * RT * CT * 2 * NT : 1];
  __shared__ float u_s[R][6];
  __shared__ float part[NW][R][4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int c = lane & 15;
  const int g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * R;

  for (int r = tid; r < R; r += NW * 64) {
    float u[6] = {0, 0, 0, 0, 0, 0};
    if (row0 + r < src.rows) row_inputs(src, net, row0 + r, u);
#pragma unroll
    for (int a = 0; a < 6; ++a) u_s[r][a] = u[a];
  }
  __syncthreads();

  // derivative factors d_l = 1 - a_l^2 of layers 1..D-1 at the wave's neurons
  DStore<P, NL, NLR, RT, CT, NT> dst;
  if constexpr (P::kBF16) {
    dst.lds = dlds;
    dst.tid = tid;
  }
  float eD[RT][CT][4];  // backward seed e_D = w_out * d_D, then e_l
  floatx4 acc[RT][CT];
  float wo[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) wo[ct] = net.wout[(wave * CT + ct) * 16 + c];

  // ---- first layer (6 -> H), FP32 vector arithmetic in the C layout
  {
    T* out_act = act[0];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n = (wave * CT + ct) * 16 + c;
      float w[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) w[a] = net.W0[n * 6 + a];
      const float b = net.bias[n];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rt * 16 + g * 4 + i;
          float z = b;
#pragma unroll
          for (int a = 0; a < 6; ++a) z += w[a] * u_s[row][a];
          float av, dv;
          tanh_d(z, av, dv);
          if (D > 1) dst.set(0, rt, ct, i, dv);
          else eD[rt][ct][i] = wo[ct] * dv;
          acc[rt][ct][i] = av;
          out_act[row * LDW + n] = (T)av;
        }
      }
    }
  }
  __syncthreads();

  // ---- hidden layers l = 1 .. D-1
  const uint4* packf = (const uint4*)net.pack_fwd;
  const uint4* packb = (const uint4*)net.pack_bwd;
  int cur = 0;
#pragma unroll
  for (int l = 1; l < D; ++l) {
    const T* in = act[cur];
    T* outp = act[NBUF == 2 ? cur ^ 1 : 0];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0, 0, 0, 0};
    const uint4* pl = packf + (size_t)(l - 1) * (H / 16) * NQ * 64;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      Pack16 a[RT], b[CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        a[rt].u = *(const uint4*)(in + (rt * 16 + c) * LDW + g * KG + q * ELEMS);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) b[ct].u = pl[((wave * CT + ct) * NQ + q) * 64 + lane];
#pragma unroll
      for (int s = 0; s < SPC; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            if constexpr (P::kBF16) {
              acc[rt][ct] = P::mma(a[rt].b, b[ct].b, acc[rt][ct]);
            } else {
              acc[rt][ct] = P::mma(a[rt].f[s], b[ct].f[s], acc[rt][ct]);
            }
          }
    }
    const float* bl = net.bias + l * H;
    if constexpr (NBUF == 1) __syncthreads();  // every wave done reading `in`
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n = (wave * CT + ct) * 16 + c;
      const float bn = bl[n];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float av, dv;
          tanh_d(acc[rt][ct][i] + bn, av, dv);
          if (l < D - 1) dst.set(l, rt, ct, i, dv);
          else eD[rt][ct][i] = wo[ct] * dv;
          acc[rt][ct][i] = av;
          outp[(rt * 16 + g * 4 + i) * LDW + n] = (T)av;
        }
    }
    __syncthreads();
    if constexpr (NBUF == 2) cur ^= 1;
  }

  // ---- output layer o = w_out . a_D + b_out
  {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float p = 0.0f;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) p += wo[ct] * acc[rt][ct][i];
        p += __shfl_xor(p, 1, 16);
        p += __shfl_xor(p, 2, 16);
        p += __shfl_xor(p, 4, 16);
        p += __shfl_xor(p, 8, 16);
        if (c == 0) part[wave][rt * 16 + g * 4 + i][0] = p;
      }
  }

  // ---- backward l = D-1 .. 1: e_l = (e_{l+1} W_l) * d_l
#pragma unroll
  for (int l = D - 1; l >= 1; --l) {
    T* eb = act[cur];
    // single buffer: every wave must be done reading the previous e_{l+2}
    if constexpr (NBUF == 1) {
      if (l < D - 1) __syncthreads();
    }
    // publish e_{l+1} at the wave's neurons
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n = (wave * CT + ct) * 16 + c;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) eb[(rt * 16 + g * 4 + i) * LDW + n] = (T)eD[rt][ct][i];
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0, 0, 0, 0};
    const uint4* pl = packb + (size_t)(l - 1) * (H / 16) * NQ * 64;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      Pack16 a[RT], b[CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        a[rt].u = *(const uint4*)(eb + (rt * 16 + c) * LDW + g * KG + q * ELEMS);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) b[ct].u = pl[((wave * CT + ct) * NQ + q) * 64 + lane];
#pragma unroll
      for (int s = 0; s < SPC; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            if constexpr (P::kBF16) {
              acc[rt][ct] = P::mma(a[rt].b, b[ct].b, acc[rt][ct]);
            } else {
              acc[rt][ct] = P::mma(a[rt].f[s], b[ct].f[s], acc[rt][ct]);
            }
          }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) eD[rt][ct][i] = acc[rt][ct][i] * dst.get(l - 1, rt, ct, i);
    // with two buffers the next layer publishes into the other one, and the
    // barrier after that write orders it after every wave's reads of this one
    if constexpr (NBUF == 2) cur ^= 1;
  }

  // ---- input gradient do/du_src = W_0[:, 0:3]^T e_1
  {
    float w[CT][3];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n = (wave * CT + ct) * 16 + c;
#pragma unroll
      for (int a = 0; a < 3; ++a) w[ct][a] = net.W0[n * 6 + a];
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float p[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int a = 0; a < 3; ++a) p[a] += w[ct][a] * eD[rt][ct][i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          p[a] += __shfl_xor(p[a], 1, 16);
          p[a] += __shfl_xor(p[a], 2, 16);
          p[a] += __shfl_xor(p[a], 4, 16);
          p[a] += __shfl_xor(p[a], 8, 16);
        }
        if (c == 0) {
          const int row = rt * 16 + g * 4 + i;
          part[wave][row][1] = p[0];
          part[wave][row][2] = p[1];
          part[wave][row][3] = p[2];
        }
      }
  }
  __syncthreads();
  for (int r = tid; r < R; r += NW * 64) {
    const int64_t row = row0 + r;
    if (row >= src.rows) continue;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      s0 += part[w][r][0];
      s1 += part[w][r][1];
      s2 += part[w][r][2];
      s3 += part[w][r][3];
    }
    RowOut o;
    o.o = s0 + net.bout;
    o.d0 = s1;
    o.d1 = s2;
    o.d2 = s3;
    out[row] = o;
  }
}

// ---------------------------------------------------------------- dispatch

template <class P, int H, int D, int NW>
hipError_t launch_one(const RowSource& src, const NetView& net, RowOut* out, hipStream_t s) {
  using Sh = Shape<P, H, D, NW>;
  const int64_t blocks = ceil_div(src.rows, Sh::R);
  hipLaunchKernelGGL((k_mlp<P, H, D, NW>), dim3((unsigned)blocks), dim3(NW * 64), 0, s, src, net,
                     out);
  return hipGetLastError();
}

template <class P>
hipError_t dispatch(int H, int D, const RowSource& src, const NetView& net, RowOut* out,
                    hipStream_t s, bool probe) {
#define SPIDER_CASE(HH, DD, NWW)                                         \
  if (H == HH && D == DD) return probe ? hipSuccess : launch_one<P, HH, DD, NWW>(src, net, out, s);
  SPIDER_CASE(32, 2, 2)
  SPIDER_CASE(32, 3, 2)
  SPIDER_CASE(32, 4, 2)
  SPIDER_CASE(64, 3, 4)
  SPIDER_CASE(64, 4, 4)
  SPIDER_CASE(128, 3, 4)
  SPIDER_CASE(128, 4, 4)
  SPIDER_CASE(128, 5, 4)
  SPIDER_CASE(256, 4, 8)
  SPIDER_CASE(256, 5, 8)
  SPIDER_CASE(256, 6, 8)
  SPIDER_CASE(256, 7, 8)
  SPIDER_CASE(256, 8, 8)
#undef SPIDER_CASE
  return hipErrorNotSupported;
}

inline uint16_t bf16_rne(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t lsb = (x >> 16) & 1u;
  return (uint16_t)((x + 0x7FFFu + lsb) >> 16);
}

template <class P>
void pack_layer(int H, const float* W, unsigned char* fwd, unsigned char* bwd) {
  using T = typename P::T;
  constexpr int ELEMS = Chunk<P>::ELEMS;
  const int NQ = chunks_per_layer<P>(H);
  const int KG = H / 4;
  const size_t esz = sizeof(T);
  for (int ct = 0; ct < H / 16; ++ct)
    for (int q = 0; q < NQ; ++q)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < ELEMS; ++e) {
          const int col = ct * 16 + (lane & 15);
          const int k = (lane >> 4) * KG + q * ELEMS + e;
          const size_t off = ((((size_t)ct * NQ + q) * 64 + lane) * ELEMS + e) * esz;
          const float vf = W[(size_t)col * H + k];  // forward: B[k][n = col] = W[n][k]
          const float vb = W[(size_t)k * H + col];  // backward: B[n = k][col] = W[n][col]
          if constexpr (P::kBF16) {
            const uint16_t a = bf16_rne(vf), b = bf16_rne(vb);
            std::memcpy(fwd + off, &a, 2);
            std::memcpy(bwd + off, &b, 2);
          } else {
            std::memcpy(fwd + off, &vf, 4);
            std::memcpy(bwd + off, &vb, 4);
          }
        }
}

}  // namespace

bool mlp_mfma_supported(int precision, int H, int D) {
  RowSource src{};
  NetView net{};
  if (precision == 1) return dispatch<PolBF16>(H, D, src, net, nullptr, 0, true) == hipSuccess;
  return dispatch<PolF32>(H, D, src, net, nullptr, 0, true) == hipSuccess;
}

size_t mfma_pack_bytes(int precision, int H) {
  return (size_t)H * H * (precision == 1 ? 2 : 4);
}

void mfma_pack_layer(int precision, int H, const float* W, void* fwd, void* bwd) {
  if (precision == 1)
    pack_layer<PolBF16>(H, W, (unsigned char*)fwd, (unsigned char*)bwd);
  else
    pack_layer<PolF32>(H, W, (unsigned char*)fwd, (unsigned char*)bwd);
}

hipError_t launch_mlp_mfma(int precision, const RowSource& src, const NetView& net, RowOut* out,
                           hipStream_t stream) {
  if (src.rows == 0) return hipSuccess;
  if (precision == 1) return dispatch<PolBF16>(net.H, net.D, src, net, out, stream, false);
  return dispatch<PolF32>(net.H, net.D, src, net, out, stream, false);
}

}  // namespace spider
