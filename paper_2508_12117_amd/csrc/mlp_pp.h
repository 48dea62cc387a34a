// Ping-pong variant of the matrix-core network kernel (BF16): the same
// forward pass and reverse-mode source gradient (Sec. 3.2) as k_mlp, with
// each wave's rows split into two halves whose layer products and epilogues
// alternate, so that one half's MFMAs run while the other half's vector
// epilogue (tanh, activation stores, derivative factors) executes.
//
// Schedule.  The layer products of a workgroup form the job sequence
//   F1A F1B F2A F2B ... F(D-1)A F(D-1)B  B(D-1)A B(D-1)B ... B1A B1B
// (F: forward hidden layer, B: backward, A/B: row half).  Phase p runs job p
// and, interleaved with its MFMAs, the epilogue of job p-1 (the first phase
// pairs F1A with the first layer of half B; the first layer of half A runs
// alone before it, the epilogue of B1B alone after the last).  A barrier
// closes every phase.  Every epilogue writes the rows of one half, which the
// job of the previous phase finished reading, while the MFMAs of the current
// phase read the other half: one activation buffer serves the whole pass.
//
// Weights.  The ring holds all chunks of the current layer's operands (both
// halves use them).  With one layer of slots, job ..B refills each chunk, as
// it frees it, with the next layer's chunk; with one and a half layers, the
// next layer's operands stream in during both jobs (see mma_half).
#pragma once
#include "mlp_mfma.h"

namespace spider {

namespace mfma {

template <class P, int H, int D, int NW, int RT_>
struct ShapePP {
  static constexpr int CT = H / 16 / NW;
  static constexpr int RT = RT_;
  static constexpr int RH = RT / 2;
  static constexpr int R = 16 * RT;
  static constexpr int NQ = chunks_per_layer<P>(H);
  static constexpr int LDW = H;
  static constexpr int CPR = H / Chunk<P>::ELEMS;
  static constexpr int SWM = CPR >= 16 ? 15 : CPR - 1;
  static constexpr int NL = D - 1;  // stored derivative layers
  static constexpr int NT = NW * 64;
  static constexpr size_t ACT_BYTES = (size_t)R * LDW * sizeof(typename P::T);
  static constexpr size_t FIXED_BYTES = (size_t)R * 8 * 4 + (size_t)(H / 16) * R * 4 * 4;
  static constexpr size_t LAYER_BYTES = (size_t)R * H * 2;
  static constexpr int LDS_LAYERS_MAX = (int)((160 * 1024 - ACT_BYTES - FIXED_BYTES) / LAYER_BYTES);
  // derivative layers go to LDS first: registers hold the weight ring
  static constexpr int NLDS = NL < LDS_LAYERS_MAX ? NL : LDS_LAYERS_MAX;
  static constexpr int NLR = NL - NLDS;
  static_assert(CT * NW * 16 == H, "H must split into 16-wide tiles over the waves");
  static_assert(RT % 2 == 0, "two row halves");
  static_assert(D >= 2, "at least one hidden layer product");
  static_assert(ACT_BYTES + FIXED_BYTES + NLDS * LAYER_BYTES <= 160 * 1024, "LDS budget");
};

// Weight ring of NS slots.  With NS = NQ (one layer), slot q holds the chunk
// of step q and half B refills it with the next layer product's chunk right
// after reading it: a whole layer's loads in every second phase.  With
// NS = 3 NQ / 2, three slot groups of NQ/2 chunks: layer product j (the j-th
// job pair of the schedule: forward layers, then backward layers) reads its
// chunks q < NQ/2 from group first(j) and the others from group second(j);
// the third group, spare(j), is free.  While job j's half A runs, the next
// product's chunks q < NQ/2 stream into spare(j); while half B runs, its
// chunks q >= NQ/2 stream into first(j), each slot refilled once half B has
// read it.  So first(j+1) = spare(j), second(j+1) = first(j) and
// spare(j+1) = second(j): the roles rotate with period three, and every phase
// issues the same number of weight loads.
__device__ __forceinline__ constexpr int ring_first(int j) { return (3 - j % 3) % 3; }
__device__ __forceinline__ constexpr int ring_slot(int j, int q, int NQ, int NS) {
  return NS == NQ ? q : ((ring_first(j) + (q < NQ / 2 ? 0 : 1)) % 3) * (NQ / 2) + q % (NQ / 2);
}

// The layer product of row half h (rows 16 (h RH + i) + c) of layer product
// j over all NQ chunks, chunk s0 + q (mod NQ) at step q, its operands in ring
// slot ring_slot(j, q).  LOADS = 1 (half A) or 2 (half B) streams the next
// layer product's operands from `next` as described above; 0 loads nothing.
// work(q) runs after the MFMAs of step q: the interleaved epilogue of the
// other half.
template <class P, int h, int RT, int CT, int NQ, int LDW, int SWM, int LOADS, int NS, class F>
__device__ __forceinline__ void mma_half(const typename P::T* X, WRing<NS, CT>& ring, int j,
                                         const WSrc& next, int voff, int c, int g, int s0,
                                         floatx4 (&acc)[RT][CT], F&& work) {
  static_assert(NS == NQ || NS == 3 * NQ / 2, "ring of one or one and a half layers");
  constexpr int RH = RT / 2, ELEMS = Chunk<P>::ELEMS, HQ = NQ / 2, ITEMS = HQ * CT;
  const typename P::T* xr = X + (h * RH * 16 + c) * LDW;
  const int sw = c & SWM;
  Pack16 x[2][RH];
#pragma unroll
  for (int i = 0; i < RH; ++i)
    x[0][i].u = *(const uint4*)(xr + i * 16 * LDW + ((4 * s0 + g) ^ sw) * ELEMS);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int b = q & 1;
    if (q + 1 < NQ) {
#pragma unroll
      for (int i = 0; i < RH; ++i)
        x[b ^ 1][i].u =
            *(const uint4*)(xr + i * 16 * LDW + ((4 * ((s0 + q + 1) & (NQ - 1)) + g) ^ sw) * ELEMS);
    }
    __builtin_amdgcn_sched_barrier(0);
    const int sq = ring_slot(j, q, NQ, NS);
#pragma unroll
    for (int i = 0; i < RH; ++i)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[h * RH + i][ct] = P::mma(ring.w[sq][ct].b, x[b][i].b, acc[h * RH + i][ct]);
    if constexpr (NS == NQ) {
      if constexpr (LOADS == 2) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) ring.w[q][ct].u = wload(next, ct * NQ + q, voff);
      }
    } else if constexpr (LOADS != 0) {
      // the ITEMS loads of this phase, spread evenly over its NQ steps: item
      // it = (chunk q' - base, tile ct) at step 2 it / CT; in half B the
      // slot of step q' - HQ has been read by then (q' - HQ <= step)
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        if (it * 2 / CT != q) continue;
        const int qn = (LOADS == 1 ? 0 : HQ) + it / CT, ct = it % CT;
        ring.w[ring_slot(j + 1, qn, NQ, NS)][ct].u = wload(next, ct * NQ + qn, voff);
      }
    }
    work(q);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Calls epi(f) for the NF epilogue fragments spread over the NQ chunk steps.
template <int NQ, int NF, class E>
__device__ __forceinline__ void spread(int q, E&& epi) {
#pragma unroll
  for (int f = 0; f < NF; ++f)
    if (f >= (q * NF) / NQ && f < ((q + 1) * NF) / NQ) epi(f);
}

template <class P, int H, int D, int NW, int RT_, int NS>
__global__ __launch_bounds__(NW * 64, 1) void k_mlp_pp(RowSource src, NetView net, RowOut* out) {
  static_assert(P::kBF16, "the ping-pong kernel is BF16 only");
  using S = ShapePP<P, H, D, NW, RT_>;
  using T = typename P::T;
  constexpr int CT = S::CT, RT = S::RT, RH = S::RH, R = S::R, NQ = S::NQ, LDW = S::LDW;
  constexpr int SWM = S::SWM, NL = S::NL, NLR = S::NLR, NT = S::NT;
  constexpr int NF = RH * CT;  // epilogue fragments per half
  constexpr int LBYTES = (H / 16) * NQ * 64 * 16;  // bytes per packed layer

  __shared__ __attribute__((aligned(16))) T act[R * LDW];
  __shared__ uint32_t dlds[S::NLDS > 0 ? S::NLDS * RT * CT * 2 * NT : 1];
  __shared__ __attribute__((aligned(16))) float u_s[R][8];
  __shared__ __attribute__((aligned(16))) float part[H / 16][R][4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform over the wave: held in a scalar register, the
  // weight-operand addresses become scalar base + per-lane offset
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15;
  const int g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * R;

  const __amdgpu_buffer_rsrc_t packf = pack_rsrc(net.pack_fwd, D - 1, LBYTES, wave * CT, NQ);
  const __amdgpu_buffer_rsrc_t packb = pack_rsrc(net.pack_bwd, D - 1, LBYTES, wave * CT, NQ);
  const int voff = lane * 16;
  WRing<NS, CT> ring;
  const int s0 = chunk_start<P, CT>(wave, NQ);
  // layer product 0 in slots 0 .. NQ-1 (groups first(0) = 0, second(0) = 1)
  ring_prime<NQ, NQ, CT>(ring, WSrc{packf, 0}, voff);
  float w1[CT][2], b1[CT][4], wo[CT][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int n0 = (wave * CT + ct) * 16 + 4 * g;
    const float4 bb = *(const float4*)(net.bias_s + n0);
    const float4 ww = *(const float4*)(net.wout + n0);
    b1[ct][0] = bb.x;
    b1[ct][1] = bb.y;
    b1[ct][2] = bb.z;
    b1[ct][3] = bb.w;
    wo[ct][0] = ww.x;
    wo[ct][1] = ww.y;
    wo[ct][2] = ww.z;
    wo[ct][3] = ww.w;
    first_layer_a(net.W0s, (wave * CT + ct) * 16 + c, g, w1[ct]);
  }

  for (int r = tid; r < R; r += NT) {
    float u[6] = {0, 0, 0, 0, 0, 0};
    if (row0 + r < src.rows) row_inputs(src, net, row0 + r, u);
#pragma unroll
    for (int a = 0; a < 6; ++a) u_s[r][a] = u[a];
    u_s[r][6] = 0.0f;
    u_s[r][7] = 0.0f;
  }
  __syncthreads();

  DStore<P, NL, NLR, RT, CT, NT> dst;
  dst.lds = dlds;
  dst.tid = tid;
  floatx4 acc[RT][CT];
  float eD[RT][CT][4];  // e_1 at the end
  float po[RT][CT];
  float u[RT][2];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    u[rt][0] = u_s[rt * 16 + c][g];
    u[rt][1] = u_s[rt * 16 + c][4 + g];
  }

  // fragment f of half h: rows 16 (h RH + f / CT) + c, neurons of tile f % CT
  auto n0_of = [&](int f) __attribute__((always_inline)) { return (wave * CT + f % CT) * 16 + 4 * g; };
  auto first_layer = [&](int h, int f) __attribute__((always_inline)) {
    const int rt = h * RH + f / CT, ct = f % CT;
    const floatx4 z = first_layer_mma(w1[ct], u[rt], b1[ct]);
    float av[4], dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) tanh_scaled(z[i], av[i], dv[i]);
    dst.set4(0, rt, ct, av, dv);
    store_row4<T>(act, LDW, SWM, rt * 16 + c, n0_of(f), av);
  };
  // epilogue of forward layer l (1 <= l <= D-1) for fragment f of half h
  auto fwd_epi = [&](int l, int h, int f) __attribute__((always_inline)) {
    const int rt = h * RH + f / CT, ct = f % CT;
    float av[4], dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) tanh_scaled(acc[rt][ct][i], av[i], dv[i]);
    if (l < D - 1) {
      dst.set4(l, rt, ct, av, dv);
      store_row4<T>(act, LDW, SWM, rt * 16 + c, n0_of(f), av);
    } else {
      // output layer partial and the backward seed e_D = w_out * d_D
      float p = wo[ct][0] * av[0], e[4];
#pragma unroll
      for (int i = 1; i < 4; ++i) p = fmaf(wo[ct][i], av[i], p);
      po[rt][ct] = p;
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i] = wo[ct][i] * dv[i];
      store_row4<T>(act, LDW, SWM, rt * 16 + c, n0_of(f), e);
    }
  };
  // epilogue of backward layer l: e_l = (e_{l+1} W_l) * d_l, published for
  // layer l-1 or kept for the input gradient
  auto bwd_epi = [&](int l, int h, int f) __attribute__((always_inline)) {
    const int rt = h * RH + f / CT, ct = f % CT;
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = dst.mul(l - 1, rt, ct, i, acc[rt][ct][i]);
    if (l > 1) {
      store_row4<T>(act, LDW, SWM, rt * 16 + c, n0_of(f), e);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) eD[rt][ct][i] = e[i];
    }
  };
  // bias of the current forward layer at the wave's neurons, loaded one
  // phase ahead of the first job that uses it
  float4 breg[CT];
  auto load_bias = [&](int l) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      breg[ct] = *(const float4*)(net.bias_s + l * H + (wave * CT + ct) * 16 + 4 * g);
  };
  auto set_bias = [&](int h) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < RH; ++i)
        acc[h * RH + i][ct] = floatx4{breg[ct].x, breg[ct].y, breg[ct].z, breg[ct].w};
  };
  load_bias(1);
  auto set_zero = [&](int h) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < RH; ++i) acc[h * RH + i][ct] = floatx4{0, 0, 0, 0};
  };

  // ---- phase 0: first layer of half A
#pragma unroll
  for (int f = 0; f < NF; ++f) first_layer(0, f);
  __syncthreads();

  // ---- forward hidden layers (layer products j = l - 1)
#pragma unroll
  for (int l = 1; l < D; ++l) {
    const int j = l - 1;
    // the next layer product: forward layer l + 1, or the last backward layer
    const WSrc pn = l < D - 1 ? WSrc{packf, l * LBYTES} : WSrc{packb, (D - 2) * LBYTES};
    // job F(l)A with the epilogue of the previous job (first layer B, or F(l-1)B)
    set_bias(0);
    mma_half<P, 0, RT, CT, NQ, LDW, SWM, 1, NS>(act, ring, j, pn, voff, c, g, s0, acc, [&](int q) {
      spread<NQ, NF>(q, [&](int f) {
        if (l == 1) first_layer(1, f);
        else fwd_epi(l - 1, 1, f);
      });
    });
    __syncthreads();
    // job F(l)B with the epilogue of F(l)A
    set_bias(1);
    if (l + 1 < D) load_bias(l + 1);
    mma_half<P, 1, RT, CT, NQ, LDW, SWM, 2, NS>(act, ring, j, pn, voff, c, g, s0, acc, [&](int q) {
      spread<NQ, NF>(q, [&](int f) { fwd_epi(l, 0, f); });
    });
    __syncthreads();
  }

  // ---- backward layers D-1 .. 1 (layer products j = 2 D - 2 - l)
#pragma unroll
  for (int l = D - 1; l >= 1; --l) {
    const int j = 2 * D - 2 - l;
    const WSrc pn{packb, (l > 1 ? l - 2 : 0) * LBYTES};
    set_zero(0);
    auto epi_a = [&](int q) {
      spread<NQ, NF>(q, [&](int f) {
        if (l == D - 1) fwd_epi(D - 1, 1, f);
        else bwd_epi(l + 1, 1, f);
      });
    };
    if (l > 1) mma_half<P, 0, RT, CT, NQ, LDW, SWM, 1, NS>(act, ring, j, pn, voff, c, g, s0, acc, epi_a);
    else mma_half<P, 0, RT, CT, NQ, LDW, SWM, 0, NS>(act, ring, j, pn, voff, c, g, s0, acc, epi_a);
    __syncthreads();
    set_zero(1);
    auto epi_b = [&](int q) { spread<NQ, NF>(q, [&](int f) { bwd_epi(l, 0, f); }); };
    if (l > 1) {
      mma_half<P, 1, RT, CT, NQ, LDW, SWM, 2, NS>(act, ring, j, pn, voff, c, g, s0, acc, epi_b);
      __syncthreads();
    } else {
      mma_half<P, 1, RT, CT, NQ, LDW, SWM, 0, NS>(act, ring, j, pn, voff, c, g, s0, acc, epi_b);
    }
  }
  // ---- epilogue of B1B
#pragma unroll
  for (int f = 0; f < NF; ++f) bwd_epi(1, 1, f);

  // ---- input gradient and output-layer partials, reduced per tile
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int n0 = (wave * CT + ct) * 16 + 4 * g;
    float w[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) w[i][a] = net.W0[(n0 + i) * 6 + a];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      float x[4];
      x[0] = po[rt][ct];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float p = w[0][a] * eD[rt][ct][0];
#pragma unroll
        for (int i = 1; i < 4; ++i) p = fmaf(w[i][a], eD[rt][ct][i], p);
        x[1 + a] = p;
      }
      part[wave * CT + ct][rt * 16 + c][g] = group_reduce_scatter(x, g);
    }
  }
  __syncthreads();
  for (int r = tid; r < R; r += NT) {
    const int64_t row = row0 + r;
    if (row >= src.rows) continue;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int tile = 0; tile < H / 16; ++tile) {
      const float4 p = *(const float4*)&part[tile][r][0];
      s0 += p.x;
      s1 += p.y;
      s2 += p.z;
      s3 += p.w;
    }
    RowOut o;
    o.o = s0 + net.bout;
    o.d0 = s1;
    o.d1 = s2;
    o.d2 = s3;
    out[row] = o;
  }
}

// NS: weight ring slots, NQ (one layer) or 3 NQ / 2
template <class P, int H, int D, int NW, int RT, int NS>
hipError_t launch_pp(const RowSource& src, const NetView& net, RowOut* out, hipStream_t s) {
  using Sh = ShapePP<P, H, D, NW, RT>;
  const int64_t blocks = ceil_div(src.rows, Sh::R);
  hipLaunchKernelGGL((k_mlp_pp<P, H, D, NW, RT, NS>), dim3((unsigned)blocks), dim3(NW * 64), 0, s,
                     src, net, out);
  return hipGetLastError();
}

}  // namespace mfma

}  // namespace spider
