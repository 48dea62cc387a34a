// Counter-based random streams of the hot path, device side.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies and xors on a 128-bit counter, key bumped by the Weyl
// constants between rounds.  Used for
//   - the minibatch permutation: a four-round Feistel network on
//     bitlength(N-1) bits whose round function is Philox word 0, with cycle
//     walking into [0, N) (minibatches without replacement, Sec. 3.2);
//   - the Langevin noise (Sec. 3.2, eq:pSGLD): two blocks per event, each
//     word pair -> a 52-bit uniform in (0, 1), Box-Muller -> two normals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spider {

constexpr uint32_t kTagNoise = 1u << 28;
constexpr uint32_t kTagPerm = 2u << 28;
constexpr int kMaxWalk = 4096;

struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Bit split of the Feistel domain [0, 2^b), b = bitlength(N - 1) (>= 1).
struct FeistelShape {
  int br;
  uint32_t mask_l, mask_r;
};

__host__ __device__ inline FeistelShape feistel_shape(int64_t N) {
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) < N) ++b;
  const int bl = b / 2;
  FeistelShape s;
  s.br = b - bl;
  s.mask_l = bl >= 32 ? 0xFFFFFFFFu : ((1u << bl) - 1u);
  s.mask_r = s.br >= 32 ? 0xFFFFFFFFu : ((1u << s.br) - 1u);
  return s;
}

__host__ __device__ inline uint64_t feistel_round4(uint64_t x, const FeistelShape& s, uint32_t k0,
                                                   uint32_t k1, uint32_t stream, uint32_t chain,
                                                   uint32_t epoch) {
  uint32_t left = (uint32_t)(x >> s.br);
  uint32_t right = (uint32_t)(x & s.mask_r);
#pragma unroll
  for (uint32_t r = 0; r < 4; ++r) {
    const uint32_t tag = kTagPerm | (stream << 4) | r;
    if ((r & 1u) == 0) {
      left ^= philox10(U4{right, epoch, chain, tag}, k0, k1).x & s.mask_l;
    } else {
      right ^= philox10(U4{left, epoch, chain, tag}, k0, k1).x & s.mask_r;
    }
  }
  return ((uint64_t)left << s.br) | right;
}

// pi(k) for k in [0, N); returns -1 if the walk cap is hit (never observed).
__host__ __device__ inline int64_t feistel_permute(int64_t k, int64_t N, const FeistelShape& s,
                                                   uint32_t k0, uint32_t k1, uint32_t stream,
                                                   uint32_t chain, uint32_t epoch) {
  uint64_t y = feistel_round4((uint64_t)k, s, k0, k1, stream, chain, epoch);
  for (int w = 0; w < kMaxWalk && y >= (uint64_t)N; ++w)
    y = feistel_round4(y, s, k0, k1, stream, chain, epoch);
  return y < (uint64_t)N ? (int64_t)y : -1;
}

__device__ inline double uniform52(uint32_t a, uint32_t b) {
  const double hi = (double)(a >> 6);
  const double lo = (double)(b >> 6);
  return (hi * 67108864.0 + lo + 0.5) * (1.0 / 4503599627370496.0);
}

// Four standard normals for event m of (stream, chain, step).
__device__ inline void noise4(uint32_t k0, uint32_t k1, uint32_t stream, uint32_t chain,
                              uint32_t step, uint32_t m, double out[4]) {
  const double two_pi = 6.283185307179586476925286766559;
#pragma unroll
  for (uint32_t sub = 0; sub < 2; ++sub) {
    const U4 w = philox10(U4{m, step, chain, kTagNoise | (stream << 4) | sub}, k0, k1);
    const double u1 = uniform52(w.x, w.y);
    const double u2 = uniform52(w.z, w.w);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(two_pi * u2, &sn, &cs);
    out[2 * sub] = rad * cs;
    out[2 * sub + 1] = rad * sn;
  }
}

}  // namespace spider
