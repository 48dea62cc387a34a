// Matrix-core travel-time network kernel template for gfx950: forward pass and
// reverse-mode source gradient (Sec. 3.2) in one launch, BF16 operands with
// FP32 accumulation (v_mfma_f32_16x16x32_bf16) or FP32 throughout
// (v_mfma_f32_16x16x4_f32).
//
// Work split.  A workgroup of NW waves handles R = 16 RT rows.  Wave w owns
// the neurons [16 CT w, 16 CT (w + 1)) of every hidden layer, in the forward
// pass and in the backward pass alike.  Every layer is computed transposed,
// neurons by rows:
//   forward   z_{l+1}[own, R] = W_l[own, H] . a_l[R, H]^T         (B from LDS)
//   backward  e_l[own, R]     = W_l[H, own]^T . e_{l+1}[R, H]^T   (B from LDS)
// so that in the accumulator layout each lane holds four consecutive neurons
// of one row.  Activations go back to LDS as one 8-byte (BF16) or 16-byte
// (FP32) store per fragment, with no exchange between lanes, and the
// derivative factors d_l = 1 - a_l^2 that the backward pass needs at its own
// neurons were produced by the same lanes in the same layout and stay on chip
// between the passes: activations are never written to memory and nothing is
// recomputed.  Hidden-layer weights stream from L2 as pre-packed A operands,
// one 16-byte coalesced load per lane per chunk.  The forward weights and
// biases carry the factor 2 log2(e) so that tanh starts from a bare base-2
// exponential.  The 6-input first layer and the 1-output last layer are FP32
// vector arithmetic on the accumulator layout.
//
// MFMA 16x16xK layouts used (lane l, c = l % 16, g = l / 16):
//   A: row c,  k-slots of group g      B: column c, k-slots of group g
//   C: column c, rows 4 g .. 4 g + 3
// with A rows = neurons, B and C columns = network rows.  Operands move in
// 16-byte chunks per lane (ELEMS elements); element j of chunk q in lane group
// g has k = (4 q + g) ELEMS + j for both operands (any consistent assignment
// gives the full dot product), so chunk q spans the 4 ELEMS consecutive
// inputs [4 q ELEMS, 4 (q + 1) ELEMS) of the layer.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace spider {

namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct PolBF16 {
  using T = __bf16;
  using V = bf16x8;                 // one MFMA operand per lane
  static constexpr int KPL = 8;     // k values per lane per MFMA
  static constexpr bool kBF16 = true;
  __device__ static floatx4 mma(const V& a, const V& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

struct PolF32 {
  using T = float;
  using V = float;
  static constexpr int KPL = 1;
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
// [neuron tile ct][chunk q][lane][ELEMS], tiles over the layer's outputs.
template <class P>
constexpr int chunks_per_layer(int H) {
  return (H / 4) / Chunk<P>::ELEMS;
}

template <class P, int H, int D, int NW, int RT_>
struct Shape {
  static constexpr int CT = H / 16 / NW;       // column tiles per wave
  static constexpr int RT = RT_;
  static constexpr int R = 16 * RT;            // rows per workgroup
  static constexpr int KG = H / 4;             // k per lane group
  static constexpr int NQ = chunks_per_layer<P>(H);
  // LDS rows of H elements, unpadded; the 16-byte chunks of row r sit at
  // chunk index ^ (r & SWM): the 16 rows that one B-operand read or fragment
  // store touches then land on 16 different chunk slots, which covers the
  // 64 banks of gfx950's LDS (with 8 slots, rows r and r + 8 collide)
  static constexpr int LDW = H;
  static constexpr int CPR = H / Chunk<P>::ELEMS;  // chunks per row
  static constexpr int SWM = CPR >= 16 ? 15 : CPR - 1;
  static constexpr int NL = D > 1 ? D - 1 : 1;  // stored derivative layers
  // derivative layers kept in registers; the rest go to LDS (BF16 pairs)
  static constexpr size_t LAYER_BYTES = (size_t)R * H * 2;  // one BF16 derivative layer
  static constexpr size_t ACT_BYTES = (size_t)R * LDW * sizeof(typename P::T);
  // row inputs [R][8] and per-tile output partials [H/16][R][4]
  static constexpr size_t UPART_BYTES = (size_t)R * 8 * 4 + (size_t)(H / 16) * R * 4 * 4;
  static constexpr int NLR_PREF = NL < 3 ? NL : 3;
  static constexpr int LDS_LAYERS_SEP = (int)((160 * 1024 - ACT_BYTES - UPART_BYTES) / LAYER_BYTES);
  // deep BF16 networks: the row inputs (dead after the first layer) and the
  // output partials (written after the backward pass) share the LDS slot of
  // derivative layer D-2 (written by forward layer D-2, last read by backward
  // layer D-1), so that one more derivative layer fits in LDS
  static constexpr bool ALIAS = P::kBF16 && D >= 3 && H * RT / NW > 64 &&
                                NL - LDS_LAYERS_SEP > NLR_PREF && LAYER_BYTES >= UPART_BYTES;
  static constexpr int LDS_LAYERS_MAX =
      ALIAS ? (int)((160 * 1024 - ACT_BYTES) / LAYER_BYTES) : LDS_LAYERS_SEP;
  static constexpr int NLR = (P::kBF16 && H * RT / NW > 64)
                                 ? (NLR_PREF > NL - LDS_LAYERS_MAX ? NLR_PREF : NL - LDS_LAYERS_MAX)
                                 : NL;
  static constexpr int NLDS = NL - NLR;
  static constexpr int NT = NW * 64;
  static constexpr size_t DLDS_BYTES = (size_t)NLDS * RT * CT * 2 * NT * 4;
  static constexpr size_t FIXED_BYTES = ALIAS ? 0 : UPART_BYTES;
  // derivative layer D-2 = NL-1 sits in LDS slot NLDS-1
  static_assert(!ALIAS || NLDS >= 1, "the shared slot must be an LDS derivative layer");
  // two activation buffers when they fit in 160 KB of LDS, else one buffer
  // and an extra barrier per layer
  static constexpr int NBUF = 2 * ACT_BYTES + DLDS_BYTES + FIXED_BYTES <= 156 * 1024 ? 2 : 1;
  static_assert(NBUF * ACT_BYTES + DLDS_BYTES + FIXED_BYTES <= 160 * 1024, "LDS budget");
  static_assert(CT * NW * 16 == H, "H must split into 16-wide tiles over the waves");
  static_assert(NQ * Chunk<P>::ELEMS == KG, "H/4 must be a whole number of chunks");
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

// tanh(z) and 1 - tanh(z)^2 from y = 2 log2(e) z (the forward weights and
// biases carry the factor): with e = 2^y = exp(2z) and r = 1/(1 + e),
// tanh z = 1 - 2r; e = inf gives +1 and e = 0 gives -1.
__device__ __forceinline__ void tanh_scaled(float y, float& a, float& d) {
  const float r = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y));
  a = fmaf(r, -2.0f, 1.0f);
  d = fmaf(-a, a, 1.0f);
}

// Derivative factors 1 - a^2 kept between the passes: FP32 registers, or in
// the BF16 path FP16 pairs (round to nearest even: 11 significant bits where
// BF16 keeps 8, and 1 - a^2 lies in [0, 1], well inside FP16's range), the
// first NLR layers in registers and the rest in LDS, where each lane reads
// back only what it wrote ([layer][pair][thread] uint32, conflict-free).  The
// backward pass multiplies by a factor with one mixed-precision FMA
// (v_fma_mix_f32 reads the FP16 half in place), mul(l, rt, ct, i, x) =
// d_l x.
// First layer (6 inputs) on the FP32 matrix core, two v_mfma_f32_16x16x4_f32
// per 16 x 16 tile: k = 0..3, then k = 4..7 with inputs 6 and 7 zero.  The
// lane supplies the A element (neuron nr = tile + lane % 16, input k = 4 kk +
// lane / 16) and the B element (row tile + lane % 16, the same k); the result
// is the accumulator layout of the hidden layers (four consecutive neurons of
// one row per lane), starting from the bias.
__device__ __forceinline__ void first_layer_a(const float* W0s, int nr, int g, float w[2]) {
  w[0] = W0s[nr * 6 + g];
  w[1] = g < 2 ? W0s[nr * 6 + 4 + g] : 0.0f;
}
__device__ __forceinline__ floatx4 first_layer_mma(const float w[2], const float u[2],
                                                   const float b[4]) {
  floatx4 z = {b[0], b[1], b[2], b[3]};
  z = __builtin_amdgcn_mfma_f32_16x16x4f32(w[0], u[0], z, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x4f32(w[1], u[1], z, 0, 0, 0);
}

template <class P, int NL, int NLR, int RT, int CT, int NT>
struct DStore {
  float v[NL][RT][CT][4];
  // a: the activations, d: their 1 - a^2 in FP32
  __device__ void set4(int l, int rt, int ct, const float a[4], const float d[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[l][rt][ct][i] = d[i];
  }
  __device__ float mul(int l, int rt, int ct, int i, float x) const { return x * v[l][rt][ct][i]; }
};

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <int NL, int NLR, int RT, int CT, int NT>
struct DStore<PolBF16, NL, NLR, RT, CT, NT> {
  uint32_t v[NLR][RT][CT][2];
  uint32_t* lds;  // [NL - NLR][RT * CT * 2][NT]
  int tid;
  // 1 - a^2 straight from the FP32 activations with one rounding to FP16
  // (v_fma_mixlo/hi_f16: fma(-a, a, 1) in full precision), written out so
  // that every tile variant rounds the same way
  __device__ void set4(int l, int rt, int ct, const float a[4], const float d[4]) {
    (void)d;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t w;
      asm("v_fma_mixlo_f16 %0, -%1, %1, 1.0 op_sel_hi:[0,0,0]\n\t"
          "v_fma_mixhi_f16 %0, -%2, %2, 1.0 op_sel_hi:[0,0,0]"
          : "=&v"(w)
          : "v"(a[2 * h]), "v"(a[2 * h + 1]));
      if (l < NLR) v[l][rt][ct][h] = w;
      else lds[(((l - NLR) * RT * CT + rt * CT + ct) * 2 + h) * NT + tid] = w;
    }
  }
  __device__ float mul(int l, int rt, int ct, int i, float x) const {
    const uint32_t w = l < NLR ? v[l][rt][ct][i >> 1]
                               : lds[(((l - NLR) * RT * CT + rt * CT + ct) * 2 + (i >> 1)) * NT + tid];
    const half2_t hv = __builtin_bit_cast(half2_t, w);
    // fma with a +0 addend (not a product, which the compiler would not fuse
    // with the conversion): d x exactly rounded, one v_fma_mix_f32
    return __builtin_fmaf((float)((i & 1) ? hv.y : hv.x), x, 0.0f);
  }
};

union Pack16 {
  uint4 u;
  bf16x8 b;
  float f[4];
};

// Element offset of (row, k) in an activation buffer: row stride ldw, 16-byte
// chunk index XOR-swizzled by the row's low bits (swm = mask).
template <class T>
__device__ __forceinline__ int act_index(int ldw, int swm, int row, int k) {
  constexpr int E = 16 / sizeof(T);
  return row * ldw + (((k / E) ^ (row & swm)) * E) + (k % E);
}

// Store the lane's accumulator fragment (four consecutive neurons n0 .. n0+3
// of one row, n0 a multiple of 4) into an activation buffer.
template <class T>
__device__ __forceinline__ void store_row4(T* buf, int ldw, int swm, int row, int n0, const float v[4]) {
  T* p = buf + act_index<T>(ldw, swm, row, n0);
  if constexpr (sizeof(T) == 2) {
    *(uint2*)p = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
  } else {
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// The four lane groups g = 0..3 of a 16-lane column each hold four partial
// sums x[0..3] (over their own four neurons of a tile).  Returns, in group g,
// component g summed over the groups as (x[0] + x[1]) + (x[2] + x[3]), the
// same order for every tile shape: two exchange steps in which each lane
// keeps half of what it still holds and sends the other half.
__device__ __forceinline__ float group_reduce_scatter(const float x[4], int g) {
  const bool b0 = g & 1, b1 = (g >> 1) & 1;
  const float keep0 = b0 ? x[1] : x[0], keep1 = b0 ? x[3] : x[2];
  const float send0 = b0 ? x[0] : x[1], send1 = b0 ? x[2] : x[3];
  const float y0 = keep0 + __shfl_xor(send0, 16);  // component b0
  const float y1 = keep1 + __shfl_xor(send1, 16);  // component b0 + 2
  const float keep = b1 ? y1 : y0, send = b1 ? y0 : y1;
  return keep + __shfl_xor(send, 32);
}

// Weight operand ring: PF chunks of the layer stream in flight per column
// tile.  The layer products of one launch (forward layers, then backward
// layers) form one stream: while a layer consumes its last chunks, the ring
// already fetches the first chunks of the next layer's operands, so their L2
// latency overlaps the epilogue and the barrier instead of stalling the next
// layer's first MFMAs.
template <int PF, int CT>
struct WRing {
  Pack16 w[PF][CT];
};

// Where a layer's packed operands come from: the pack as a buffer resource
// (scalar base and range) and the layer's byte offset in it.  A 16-byte
// chunk is then a buffer load with a scalar offset (layer, tile, chunk: all
// uniform over the wave) and the lane's fixed 16-byte slot, so the weight
// stream costs no per-lane address arithmetic.
struct WSrc {
  __amdgpu_buffer_rsrc_t rsrc;
  int32_t off;
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The pack of `layers` hidden layers at p as a buffer resource.
// The resource covers the wave's own column tiles only: it starts at tile
// wave_tile0 (tiles of NQ 1 KB chunks), so that every operand offset below
// is a compile-time constant.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pack_rsrc(const void* p, int layers,
                                                           int layer_bytes, int wave_tile0,
                                                           int NQ) {
  const int skip = wave_tile0 * NQ * 1024;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>((const char*)p + skip), 0,
                                           layers * layer_bytes - skip, 0x00020000);
}

// Chunk `chunk` (index ct * NQ + position within the wave's tile ct; the
// packing stores a tile's chunks in the order the kernels use them) of a
// layer, this lane's 16 bytes (voff = 16 lane).
__device__ __forceinline__ uint4 wload(const WSrc& s, int chunk, int voff) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(s.rsrc, voff, s.off + chunk * 1024, 0);
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Order of the K chunks.  BF16 products add their chunks starting at the
// chunk of the output neuron's own 32-neuron block (n / 32) and wrapping
// around, so that a wave can begin with the chunk it produced itself; the
// order depends on the neuron only, so every tile variant adds in the same
// order (waves own at most one 32-neuron block: CT <= 2).  FP32 products add
// chunks in index order.  The packs store each column tile's chunks in this
// order (tile_chunk_start).
__host__ __device__ constexpr int tile_chunk_start(bool bf16, int tile, int NQ) {
  return bf16 ? (tile / 2) & (NQ - 1) : 0;
}
template <class P, int CT>
__device__ __forceinline__ int chunk_start(int wave, int NQ) {
  static_assert(!P::kBF16 || CT <= 2, "a wave's neurons lie in one 32-neuron block");
  return tile_chunk_start(P::kBF16, wave * CT, NQ);
}

// Prefetch ring slots j = 0 .. PF-1 with the first PF chunks (in the order
// of use) of pl.
template <int NQ, int PF, int CT, int SLOTS>
__device__ __forceinline__ void ring_prime(WRing<SLOTS, CT>& r, const WSrc& pl, int voff) {
  static_assert(PF <= SLOTS, "ring too small");
#pragma unroll
  for (int j = 0; j < PF; ++j)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) r.w[j][ct].u = wload(pl, ct * NQ + j, voff);
}

// acc[rt][ct] += W[neuron tile wave*CT + ct][k] . X[16 rt + row][k] over the
// layer's K = H, chunks in the order s0, s0 + 1, ... (mod NQ): the weights
// are the A operand, taken from the ring (processing step q in slot q % PF),
// which is refilled PF steps ahead from pl and then from pl_next (for the
// last layer of the launch pass pl again: the refill is then unused); the
// rows X are the B operand, read from LDS (row stride LDW, swizzled chunks)
// one chunk ahead of the MFMAs that use them.  Every load is issued without
// a branch around it, so the wait counts stay exact and the ring keeps PF
// chunks in flight.
template <class P, int RT, int CT, int NQ, int LDW, int SWM, int PF>
__device__ __forceinline__ void layer_mma(const typename P::T* X, const WSrc& pl,
                                          const WSrc& pl_next, WRing<PF, CT>& ring, int voff,
                                          int c, int g, int s0, floatx4 (&acc)[RT][CT]) {
  constexpr int ELEMS = Chunk<P>::ELEMS, SPC = Chunk<P>::SPC;
  static_assert(NQ % PF == 0, "chunks must split evenly over the prefetch ring");
  static_assert(PF % 2 == 0 || PF == NQ, "the B double buffer alternates with the chunk parity");
  static_assert((NQ & (NQ - 1)) == 0, "chunks per lane group must be a power of two");
  // rows 16 rt + c share the swizzle c & SWM (SWM < 16)
  const typename P::T* xr = X + c * LDW;
  const int sw = c & SWM;
  Pack16 x[2][RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
    x[0][rt].u = *(const uint4*)(xr + rt * 16 * LDW + ((4 * s0 + g) ^ sw) * ELEMS);
#pragma unroll 1
  for (int q0 = 0; q0 < NQ; q0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int q = q0 + j;
      const int b = j & 1;  // q0 is even whenever PF < NQ
      // next chunk (after the last one the first again: an unused read)
      const int qn = (s0 + q + 1) & (NQ - 1);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        x[b ^ 1][rt].u = *(const uint4*)(xr + rt * 16 * LDW + ((4 * qn + g) ^ sw) * ELEMS);
      __builtin_amdgcn_sched_barrier(0);  // issue them before this chunk's MFMAs
#pragma unroll
      for (int s = 0; s < SPC; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            if constexpr (P::kBF16) {
              acc[rt][ct] = P::mma(ring.w[j][ct].b, x[b][rt].b, acc[rt][ct]);
            } else {
              acc[rt][ct] = P::mma(ring.w[j][ct].f[s], x[b][rt].f[s], acc[rt][ct]);
            }
          }
      const bool here = q + PF < NQ;
      const WSrc src = here ? pl : pl_next;
      const int qc = (q + PF) & (NQ - 1);  // position in the order of use
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) ring.w[j][ct].u = wload(src, ct * NQ + qc, voff);
      // keep the refill here, right after the MFMAs that free the slot
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// MINB workgroups per CU are targeted (MINB = 2 asks the compiler for at most
// 256 registers per wave so that two independent workgroups share each SIMD
// and one's vector epilogue overlaps the other's matrix work).
template <class P, int H, int D, int NW, int RT_, int PF = 4, int MINB = 1>
__global__ __launch_bounds__(NW * 64, MINB) void k_mlp(RowSource src, NetView net, RowOut* out) {
  using S = Shape<P, H, D, NW, RT_>;
  using T = typename P::T;
  constexpr int CT = S::CT, RT = S::RT, R = S::R, NQ = S::NQ, LDW = S::LDW, SWM = S::SWM;
  constexpr int NL = S::NL, NLR = S::NLR, NT = S::NT, NBUF = S::NBUF;

  __shared__ __attribute__((aligned(16))) T act[NBUF][R * LDW];
  __shared__ __attribute__((aligned(16))) uint32_t dlds[S::NLDS > 0 ? S::NLDS * RT * CT * 2 * NT : 1];
  __shared__ __attribute__((aligned(16))) float upart_own[S::ALIAS ? 4 : S::UPART_BYTES / 4];
  float* upart = S::ALIAS ? (float*)(dlds + (size_t)(S::NLDS - 1) * RT * CT * 2 * NT) : upart_own;
  // row inputs, then (after the backward pass) the per 16-neuron tile partial
  // sums of the output layer and the input gradient; summed over tiles in a
  // fixed order, so the result does not depend on how the tiles are split
  // over the waves
  float (*u_s)[8] = (float (*)[8])upart;
  float (*part)[R][4] = (float (*)[R][4])(upart + R * 8);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform over the wave: held in a scalar register, the
  // weight-operand addresses become scalar base + per-lane offset
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15;
  const int g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * R;

  // hidden-layer operand stream: forward layers 1 .. D-1, then backward
  // layers D-1 .. 1; the ring starts filling now, under the first layer
  constexpr int LBYTES = (H / 16) * NQ * 64 * 16;  // bytes per packed layer
  constexpr int NLAY = D > 1 ? D - 1 : 1;
  const __amdgpu_buffer_rsrc_t packf = pack_rsrc(net.pack_fwd, NLAY, LBYTES, wave * CT, NQ);
  const __amdgpu_buffer_rsrc_t packb = pack_rsrc(net.pack_bwd, NLAY, LBYTES, wave * CT, NQ);
  const int voff = lane * 16;
  constexpr int PFR = NQ < PF ? NQ : PF;
  WRing<PFR, CT> ring;
  const int s0 = chunk_start<P, CT>(wave, NQ);
  if (D > 1) ring_prime<NQ, PFR, CT>(ring, WSrc{packf, 0}, voff);
  // first-layer and output weights of the wave's neurons, loaded before the
  // row inputs so that both latencies overlap
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

  for (int r = tid; r < R; r += NW * 64) {
    float u[6] = {0, 0, 0, 0, 0, 0};
    if (row0 + r < src.rows) row_inputs(src, net, row0 + r, u);
#pragma unroll
    for (int a = 0; a < 6; ++a) u_s[r][a] = u[a];
    u_s[r][6] = 0.0f;
    u_s[r][7] = 0.0f;
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
  float po[RT][CT];     // output layer over the lane's four neurons of a tile

  // ---- first layer (6 -> H) in FP32 on the matrix core, into the C layout
  {
    float u[RT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      u[rt][0] = u_s[rt * 16 + c][g];
      u[rt][1] = u_s[rt * 16 + c][4 + g];
    }
    T* out_act = act[0];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n0 = (wave * CT + ct) * 16 + 4 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const floatx4 z = first_layer_mma(w1[ct], u[rt], b1[ct]);
        float av[4], dv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          tanh_scaled(z[i], av[i], dv[i]);
          if (D == 1) eD[rt][ct][i] = wo[ct][i] * dv[i];
          acc[rt][ct][i] = av[i];
        }
        if (D > 1) {
          dst.set4(0, rt, ct, av, dv);
          store_row4<T>(out_act, LDW, SWM, rt * 16 + c, n0, av);
        }
      }
    }
  }
  if (D > 1) __syncthreads();

  // ---- hidden layers l = 1 .. D-1; the last one's activations feed only the
  // output layer, from registers
  int cur = 0;
#pragma unroll
  for (int l = 1; l < D; ++l) {
    const T* in = act[cur];
    T* outp = act[NBUF == 2 ? cur ^ 1 : 0];
    // the accumulators start from the bias: z = b + W a
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float4 bn = *(const float4*)(net.bias_s + l * H + (wave * CT + ct) * 16 + 4 * g);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = floatx4{bn.x, bn.y, bn.z, bn.w};
    }
    const WSrc pl{packf, (l - 1) * LBYTES};
    const WSrc pn = l < D - 1 ? WSrc{packf, l * LBYTES} : WSrc{packb, (D - 2) * LBYTES};
    layer_mma<P, RT, CT, NQ, LDW, SWM, PFR>(in, pl, pn, ring, voff, c, g, s0, acc);
    if constexpr (NBUF == 1) __syncthreads();  // every wave done reading `in`
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int n0 = (wave * CT + ct) * 16 + 4 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        float av[4], dv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          tanh_scaled(acc[rt][ct][i], av[i], dv[i]);
          if (l == D - 1) eD[rt][ct][i] = wo[ct][i] * dv[i];
          acc[rt][ct][i] = av[i];
        }
        if (l < D - 1) {
          dst.set4(l, rt, ct, av, dv);
          store_row4<T>(outp, LDW, SWM, rt * 16 + c, n0, av);
        }
      }
    }
    if (l < D - 1) __syncthreads();
    if constexpr (NBUF == 2) cur ^= 1;
  }

  // ---- output layer o = w_out . a_D + b_out, the lane's four neurons
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      float p = wo[ct][0] * acc[rt][ct][0];
#pragma unroll
      for (int i = 1; i < 4; ++i) p = fmaf(wo[ct][i], acc[rt][ct][i], p);
      po[rt][ct] = p;
    }

  // source columns of W_0 for the input gradient, loaded ahead of the
  // backward pass
  float wg[CT][4][3];

  // ---- backward l = D-1 .. 1: e_l = (e_{l+1} W_l) * d_l.  With two buffers
  // the first write goes to the one that layer D-2 read, which every wave
  // finished before the barrier that closed that layer.
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
      const int n0 = (wave * CT + ct) * 16 + 4 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) store_row4<T>(eb, LDW, SWM, rt * 16 + c, n0, eD[rt][ct]);
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0, 0, 0, 0};
    const WSrc pl{packb, (l - 1) * LBYTES};
    const WSrc pn = l > 1 ? WSrc{packb, (l - 2) * LBYTES} : pl;
    if (l == 1) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int n0 = (wave * CT + ct) * 16 + 4 * g;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int a = 0; a < 3; ++a) wg[ct][i][a] = net.W0[(n0 + i) * 6 + a];
      }
    }
    layer_mma<P, RT, CT, NQ, LDW, SWM, PFR>(eb, pl, pn, ring, voff, c, g, s0, acc);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) eD[rt][ct][i] = dst.mul(l - 1, rt, ct, i, acc[rt][ct][i]);
    // with two buffers the next layer publishes into the other one, and the
    // barrier after that write orders it after every wave's reads of this one
    if constexpr (NBUF == 2) cur ^= 1;
  }

  // ---- input gradient do/du_src = W_0[:, 0:3]^T e_1, with the output layer
  // partial, reduced over each tile's 16 neurons
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const float (&w)[4][3] = wg[ct];
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
  for (int r = tid; r < R; r += NW * 64) {
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

// ---------------------------------------------------------------- launch

template <class P, int H, int D, int NW, int RT, int PF = 4, int MINB = 1>
hipError_t launch_variant(const RowSource& src, const NetView& net, RowOut* out, hipStream_t s) {
  using Sh = Shape<P, H, D, NW, RT>;
  const int64_t blocks = ceil_div(src.rows, Sh::R);
  hipLaunchKernelGGL((k_mlp<P, H, D, NW, RT, PF, MINB>), dim3((unsigned)blocks), dim3(NW * 64), 0,
                     s, src, net, out);
  return hipGetLastError();
}

inline uint16_t bf16_rne(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t lsb = (x >> 16) & 1u;
  return (uint16_t)((x + 0x7FFFu + lsb) >> 16);
}

// Host-side packing of one hidden layer into the operand order above; the
// forward operand holds fscale W (the tanh argument scale), rounded once.
template <class P>
void pack_layer(int H, const float* W, double fscale, unsigned char* fwd, unsigned char* bwd) {
  using T = typename P::T;
  constexpr int ELEMS = Chunk<P>::ELEMS;
  const int NQ = chunks_per_layer<P>(H);
  const size_t esz = sizeof(T);
  for (int ct = 0; ct < H / 16; ++ct)
    for (int pos = 0; pos < NQ; ++pos)  // position pos holds the chunk used pos-th
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < ELEMS; ++e) {
          const int q = (tile_chunk_start(P::kBF16, ct, NQ) + pos) & (NQ - 1);
          const int n = ct * 16 + (lane & 15);
          const int k = (4 * q + (lane >> 4)) * ELEMS + e;
          const size_t off = ((((size_t)ct * NQ + pos) * 64 + lane) * ELEMS + e) * esz;
          // forward: A[n][k] = W[n][k]; backward: A[n][k] = W[k][n]
          const float vf = (float)(fscale * (double)W[(size_t)n * H + k]);
          const float vb = W[(size_t)k * H + n];
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

}  // namespace mfma

}  // namespace spider
