// Per-step kernels of the minibatch pipeline around the travel-time network.
//
//   select    minibatch without replacement (Sec. 3.2) and its gathers; each
//             entry (events i and j of an observation) is counted under its
//             (chain, event) key with an arrival rank
//   csr       exclusive scan of the counts, scatter of the entries to their
//             key's segment, and each segment sorted by (group, entry): a
//             fixed order whatever the ranks were, in which the entries of a
//             (chain, group, event) node of the whitening are contiguous
//   assemble  T and dT/dx in FP64 from the network outputs; the network runs
//             over the rows in CSR order, so dT/dx lands in CSR order
//   residual  r = tau - [T_i - T_j + t_i - t_j] (Eq. 1); whitening in closed
//             form where it applies: z = r / sigma^2 (none), r / (sigma^2 +
//             2 kappa^2 w) (diagonal, and exact for an observation whose two
//             nodes hold only it), sign(r) (the L1 loss of Stage 1)
//   whitening exact Sigma_B^{-1} r (Sec. 3.1, eq:marginal_sigma) for the
//             other observations: by Woodbury, z = (r - U y)/sigma^2 with
//             (lambda I + U^T U) y = U^T r per (chain, group) system, solved
//             by leaf elimination and CG on the cyclic core; the solver
//             writes z at both entries of each of its observations
//   reduce    per-event gradient (eq:sgd): the sum over one CSR segment per
//             (chain, event), in CSR order
// No floating-point atomics anywhere: every sum runs in a fixed order, so a
// step is bitwise reproducible.
#include <cstdlib>

#include "device_rng.h"
#include "internal.h"
#include "tt_assemble.h"

namespace spider {

namespace {

constexpr int kBlock = 256;
constexpr int kWhitenExact = 2;  // SPIDER_WHITEN_EXACT
constexpr int32_t kSingle = (int32_t)0x80000000;  // pos bit: the node holds one entry
constexpr int32_t kPosMask = 0x7fffffff;

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = ceil_div(n, block);
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Sum of one double per thread over the block, the same fixed tree every
// time: butterfly within each wave, then the wave sums in wave order (every
// thread returns the sum).  sh holds TB / 64 doubles.
template <int TB>
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < TB / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- scan

constexpr int kScanTB = 256;
constexpr int kScanIPT = 16;                     // items per thread
constexpr int kScanChunk = kScanTB * kScanIPT;  // items per block

// Inclusive block scan of one value per thread (fixed order).
__device__ inline int32_t block_scan_incl(int32_t v, int32_t* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanTB; d <<= 1) {
    const int32_t x = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const int32_t r = sh[t];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanTB) void k_scan_reduce(const int32_t* a, int64_t len,
                                                         int32_t* part) {
  __shared__ int32_t sh[kScanTB];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanIPT;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i)
    if (base + i < len) s += a[base + i];
  s = block_scan_incl(s, sh);
  if (threadIdx.x == kScanTB - 1) part[blockIdx.x] = s;
}

// Exclusive scan of the block sums by one block.
__global__ __launch_bounds__(kScanTB) void k_scan_top(int32_t* part, int64_t nb) {
  __shared__ int32_t sh[kScanTB];
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanTB) {
    const int64_t k = b0 + threadIdx.x;
    const int32_t v = k < nb ? part[k] : 0;
    const int32_t incl = block_scan_incl(v, sh);
    if (k < nb) part[k] = carry + incl - v;
    carry += sh[kScanTB - 1];  // this chunk's total (sh still holds the scan)
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanTB) void k_scan_apply(int32_t* a, int64_t len,
                                                        const int32_t* part) {
  __shared__ int32_t sh[kScanTB];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanIPT;
  int32_t v[kScanIPT];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    v[i] = base + i < len ? a[base + i] : 0;
    s += v[i];
  }
  const int32_t incl = block_scan_incl(s, sh);
  int32_t run = part[blockIdx.x] + incl - s;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    if (base + i < len) a[base + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------- select

__global__ void k_select(CatView cat, int C, int64_t n, const int64_t* idx, uint32_t k0,
                         uint32_t k1, const int64_t* steps, int64_t step_scalar, int chain0,
                         BatchBufs b, int* err) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)C * n) return;
  const int c = (int)(q / n);
  const int64_t k = q - (int64_t)c * n;
  int64_t o;
  if (idx) {
    o = idx[k];
  } else {
    const int64_t t = (steps ? steps[c] : 0) + step_scalar;
    const int64_t B = cat.N / n;
    const int64_t epoch = t / B;
    const int64_t j = t - epoch * B;
    const FeistelShape sh = feistel_shape(cat.N);
    o = feistel_permute(j * n + k, cat.N, sh, k0, k1, cat.stream, (uint32_t)(chain0 + c),
                        (uint32_t)epoch);
  }
  if (o < 0 || o >= cat.N) {
    atomicOr(err, kErrSelect);
    o = 0;
  }
  const ObsRec rc = cat.rec[o];
  if (b.obs) b.obs[q] = o;
  b.ev[2 * q] = rc.i;
  b.ev[2 * q + 1] = rc.j;
  b.sta[2 * q] = rc.g;
  b.sta[2 * q + 1] = rc.g;
  b.tau[q] = (double)rc.dt;
  b.w[q] = rc.w;
}

// ---------------------------------------------------------------- CSR

// Sort key of an entry inside its event's segment: (group, entry).
// ---------------------------------------------------------------- CSR build
//
// The CSR order is unique: chain, then event, then (group, entry) within the
// event.  Entries are first gathered into buckets of (chain, block of 2^sb
// consecutive events), bucket-major: a counting pass histograms the buckets
// in LDS per block of kBucketHB entries, a prefix over those blocks and a scan
// of the bucket totals give every (bucket, block) its first slot, and a
// scatter pass appends each entry's record there (LDS atomics decide the
// order within a block, which the next pass erases).  One workgroup per
// bucket then orders the bucket in LDS: counting sort by event, each event's
// segment by (group, entry), and writes the CSR arrays; nothing depends on
// the arrival order, and no global atomics are used.

constexpr int64_t kBucketHB = 65536;  // entries per counting block (within one chain)
constexpr int kBucketTB = 1024;       // threads of the counting and scatter blocks
constexpr int kBucketU = 8;           // entries per thread whose loads are in flight together
constexpr int64_t kBucketMax = 16384; // buckets per chain (LDS counters)
constexpr int kBucketMaxSB = 13;      // at most 8,192 events per bucket
constexpr int kSortTB = 512;          // threads per bucket
constexpr int64_t kBucketTarget = 4096;  // average records per bucket aimed at

// A record: event within its bucket (bits 48..60), group (32..47), entry.
__device__ inline uint64_t bucket_record(int32_t m_local, int32_t g, int32_t e) {
  return ((uint64_t)(uint32_t)m_local << 48) | ((uint64_t)(uint32_t)g << 32) | (uint32_t)e;
}

// Block (j, c) of the counting and scatter passes: entries [2 n c + j HB,
// ...) of chain c; its counts at counts[(c hbc + j) nbk + k] for the chain's
// buckets k.
__global__ __launch_bounds__(kBucketTB) void k_bucket_count(int64_t n, int sb, int64_t nbk,
                                                           const int32_t* ev, int32_t* counts) {
  extern __shared__ int32_t h[];
  for (int64_t k = threadIdx.x; k < nbk; k += kBucketTB) h[k] = 0;
  __syncthreads();
  const int64_t c = blockIdx.y;
  const int64_t e0 = 2 * n * c + (int64_t)blockIdx.x * kBucketHB;
  const int64_t e1 = min(2 * n * (c + 1), e0 + kBucketHB);
  // kBucketU entries per thread at a time, their loads issued together
  for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)kBucketTB * kBucketU) {
    int32_t m[kBucketU];
#pragma unroll
    for (int u = 0; u < kBucketU; ++u) {
      const int64_t x = e + u * kBucketTB;
      m[u] = x < e1 ? ev[x] : -1;
    }
#pragma unroll
    for (int u = 0; u < kBucketU; ++u)
      if (m[u] >= 0) atomicAdd(&h[m[u] >> sb], 1);
  }
  __syncthreads();
  int32_t* row = counts + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nbk;
  for (int64_t k = threadIdx.x; k < nbk; k += kBucketTB) row[k] = h[k];
}

// Per bucket (chain c, block k of events): the counts of the chain's
// counting blocks become offsets within the bucket (in block order) and the
// bucket total goes to tot[c nbk + k]; tot[nb] = 0 and start[keys] = E for
// what follows.
__global__ void k_bucket_prefix(int64_t nbk, int64_t nb, int64_t hbc, int32_t* counts,
                                int32_t* tot, int32_t* start, int64_t keys, int64_t E) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id == 0) {
    tot[nb] = 0;
    start[keys] = (int32_t)E;
  }
  if (id >= nb) return;
  const int64_t c = id / nbk, k = id - c * nbk;
  int32_t* col = counts + c * hbc * nbk + k;
  int32_t run = 0;
  for (int64_t j = 0; j < hbc; ++j) {
    const int32_t x = col[j * nbk];
    col[j * nbk] = run;
    run += x;
  }
  tot[id] = run;
}

__global__ __launch_bounds__(kBucketTB) void k_bucket_scatter(int64_t n, int sb, int64_t nbk,
                                                             const int32_t* counts,
                                                             const int32_t* base, BatchBufs b) {
  extern __shared__ int32_t cur[];
  const int64_t c = blockIdx.y;
  const int32_t* row = counts + (c * gridDim.x + blockIdx.x) * nbk;
  const int32_t* bb = base + c * nbk;
  for (int64_t k = threadIdx.x; k < nbk; k += kBucketTB) cur[k] = bb[k] + row[k];
  __syncthreads();
  const int64_t e0 = 2 * n * c + (int64_t)blockIdx.x * kBucketHB;
  const int64_t e1 = min(2 * n * (c + 1), e0 + kBucketHB);
  const int32_t mask = (1 << sb) - 1;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)kBucketTB * kBucketU) {
    int32_t m[kBucketU], g[kBucketU];
#pragma unroll
    for (int u = 0; u < kBucketU; ++u) {
      const int64_t x = e + u * kBucketTB;
      m[u] = -1;
      if (x < e1) {
        m[u] = b.ev[x];
        g[u] = b.sta[x];
      }
    }
#pragma unroll
    for (int u = 0; u < kBucketU; ++u) {
      if (m[u] < 0) continue;
      const int32_t slot = atomicAdd(&cur[m[u] >> sb], 1);
      b.ckey[slot] = bucket_record(m[u] & mask, g[u], (int32_t)(e + u * kBucketTB));
    }
  }
}

// Ascending sort network for any length len (positions at or past len act as
// +infinity, so comparators that touch them are skipped): bitonic stages in
// which the first step of each merge compares mirrored pairs.  get/put are
// the element accessors; all threads of the block call it.
template <class Get, class Put>
__device__ void block_sort_any(int32_t len, Get&& get, Put&& put) {
  int32_t P2 = 1;
  while (P2 < len) P2 <<= 1;
  for (int32_t kk = 2; kk <= P2; kk <<= 1) {
    for (int32_t i = threadIdx.x; i < P2 / 2; i += blockDim.x) {
      const int32_t half = kk >> 1, blk = i / half, off = i % half;
      const int32_t a = blk * kk + off, c = blk * kk + kk - 1 - off;
      if (c < len) {
        const uint64_t x = get(a), y = get(c);
        if (x > y) {
          put(a, y);
          put(c, x);
        }
      }
    }
    __syncthreads();
    for (int32_t j = kk >> 2; j >= 1; j >>= 1) {
      for (int32_t i = threadIdx.x; i < P2 / 2; i += blockDim.x) {
        const int32_t a = (i / j) * 2 * j + i % j, c = a + j;
        if (c < len) {
          const uint64_t x = get(a), y = get(c);
          if (x > y) {
            put(a, y);
            put(c, x);
          }
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per bucket: the bucket's records in (event, group, entry)
// order, then per position the entry (csr), its event and group, its node's
// first position with the single-entry bit (hd) and, at that position, one
// past the node's last (nend), all written in CSR order; start[] of the
// bucket's events.  A bucket of up to cap records (held in registers after
// one read) is ordered in LDS: by a counting sort on the event (placement
// order within an event from LDS atomics), then each event's segment by
// every record's rank within it.  A larger bucket is sorted in place in
// global memory by a sort network.
// Dynamic LDS: cap records, then 2 (2^sb + 1) ints.
template <int RPT>  // records per thread held in registers: cap = RPT kSortTB
__global__ __launch_bounds__(kSortTB) void k_bucket_sort(int64_t nbk, int sb, int M,
                                                        const int32_t* base, BatchBufs b) {
  constexpr int cap = RPT * kSortTB;
  extern __shared__ uint64_t dyn[];
  uint64_t* k_sh = dyn;
  int32_t* soff = (int32_t*)(dyn + cap);  // [2^sb + 1] offsets, then cursors
  int32_t* cur = soff + (1 << sb) + 1;
  __shared__ int32_t wsum[kSortTB / 64];
  const int t = threadIdx.x;
  const int64_t bk = blockIdx.x;
  const int64_t c = bk / nbk;
  const int32_t m0 = (int32_t)((bk - c * nbk) << sb);
  const int32_t nev = min(1 << sb, M - m0);
  const int32_t r0 = base[bk], len = base[bk + 1] - r0;
  uint64_t* rec = b.ckey + r0;
  const bool in_lds = len <= cap;

  uint64_t reg[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int32_t i = t + u * kSortTB;
    reg[u] = (in_lds && i < len) ? rec[i] : 0;
  }
  for (int32_t m = t; m <= nev; m += kSortTB) soff[m] = 0;
  __syncthreads();
  if (in_lds) {
#pragma unroll
    for (int u = 0; u < RPT; ++u)
      if (t + u * kSortTB < len) atomicAdd(&soff[(int32_t)(reg[u] >> 48)], 1);
  } else {
    for (int32_t i = t; i < len; i += kSortTB) atomicAdd(&soff[(int32_t)(rec[i] >> 48)], 1);
  }
  __syncthreads();
  // ---- segment offsets (exclusive scan over contiguous chunks, wave scans,
  // wave totals) and start[] of the bucket's events
  {
    const int lane = t & 63, w = t >> 6;
    const int32_t per = (nev + kSortTB - 1) / kSortTB;
    const int32_t k0 = t * per, k1 = min(nev, k0 + per);
    int32_t cnt = 0;
    for (int32_t k = k0; k < k1; ++k) cnt += soff[k];
    int32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t before = 0;
#pragma unroll
    for (int v = 0; v < kSortTB / 64; ++v)
      if (v < w) before += wsum[v];
    int32_t o = before + incl - cnt;
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t x = soff[k];
      soff[k] = o;
      cur[k] = o;
      o += x;
    }
    if (t == 0) soff[nev] = len;
  }
  __syncthreads();
  int32_t* key_start = b.start + c * M + m0;
  for (int32_t m = t; m < nev; m += kSortTB) key_start[m] = r0 + soff[m];

  // ---- the order
  if (in_lds) {
#pragma unroll
    for (int u = 0; u < RPT; ++u)
      if (t + u * kSortTB < len) k_sh[atomicAdd(&cur[(int32_t)(reg[u] >> 48)], 1)] = reg[u];
    __syncthreads();
    // each segment in (group, entry) order: every record's rank among its
    // segment's (the records are distinct: they hold the entry), then each
    // moves to its rank (every record ranks itself, all in parallel)
    int32_t dst[RPT];
    uint64_t val[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int32_t i = t + u * kSortTB;
      dst[u] = -1;
      val[u] = 0;
      if (i >= len) continue;
      const uint64_t x = k_sh[i];
      const int32_t m = (int32_t)(x >> 48);
      const int32_t p0 = soff[m], p1 = soff[m + 1];
      if (p1 - p0 == 1) continue;
      int32_t rank = 0;
      for (int32_t j = p0; j < p1; ++j) rank += k_sh[j] < x ? 1 : 0;
      dst[u] = p0 + rank;
      val[u] = x;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u)
      if (dst[u] >= 0) k_sh[dst[u]] = val[u];
  } else {
    block_sort_any(len, [&](int32_t i) { return rec[i]; }, [&](int32_t i, uint64_t x) { rec[i] = x; });
  }
  __syncthreads();

  // ---- per position: node runs are the positions of equal (event, group)
  auto key_at = [&](int32_t i) { return in_lds ? k_sh[i] : rec[i]; };
  for (int32_t i = t; i < len; i += kSortTB) {
    const uint64_t x = key_at(i);
    const uint64_t eg = x >> 32;  // (event, group)
    int32_t j = i;
    while (j > 0 && (key_at(j - 1) >> 32) == eg) --j;
    const bool last = i + 1 == len || (key_at(i + 1) >> 32) != eg;
    const int32_t p = r0 + i, e = (int32_t)(uint32_t)x;
    b.csr[p] = e;
    b.pev[p] = m0 + (int32_t)(x >> 48);
    b.pgr[p] = (int32_t)(eg & 0xFFFF);
    b.hd[p] = (r0 + j) | ((last && j == i) ? kSingle : 0);
    if (last) b.nend[r0 + j] = p + 1;
  }
}

// ---------------------------------------------------------------- two phases

__global__ void k_phase_flags(int64_t E, BatchBufs b, int32_t L_p, int32_t* flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > E) return;
  flags[p] = p < E && b.pgr[p] < L_p ? 1 : 0;
}

// After the exclusive scan of the flags: the positions of P entries at their
// rank, those of S entries after all P ones, both in CSR order; flags[E] =
// the P count.
__global__ void k_phase_rows(int64_t E, BatchBufs b, int32_t L_p, const int32_t* flags,
                             int64_t* n_p) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= E) return;
  const int32_t np = flags[E];
  const int32_t rp = flags[p];
  if (b.pgr[p] < L_p) b.rows[rp] = (int32_t)p;
  else b.rows[np + (int32_t)(p - rp)] = (int32_t)p;
  if (p == 0) *n_p = np;
}

// ---------------------------------------------------------------- assemble

__global__ void k_assemble(CatView cat, NetView net, NetView net_s, int64_t n, const double* theta,
                           int64_t theta_stride, const int32_t* rows, int64_t E, BatchBufs b,
                           bool grad64, int32_t* act_clear) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= E) return;
  if (act_clear) act_clear[v] = 0;  // the exact whitening's node flags, set by k_residual
  const int32_t p = rows ? rows[v] : (int32_t)v;
  const int32_t e = b.csr[p];
  const int64_t c = p / (2 * n);  // chain c holds positions [2 n c, 2 n (c + 1))
  const int32_t g = b.pgr[p];
  const double4 xe = *(const double4*)(theta + c * theta_stride + (int64_t)b.pev[p] * 4);
  const double* st = cat.stations + (int64_t)g * 3;
  const double x[3] = {xe.x, xe.y, xe.z};
  const double s[3] = {st[0], st[1], st[2]};
  double T, gr[3];
  assemble_tt(g >= cat.L_p ? net_s : net, x, s, b.net_out[v], T, gr);
  const int32_t h = b.hd[p];
  TRec o;
  o.T = T + xe.w;  // with the event's origin time, for the residual
  o.p = p | (h & kSingle);
  o.head = h & kPosMask;
  b.tr[e] = o;
  if (grad64) {
    b.gT64[(int64_t)p * 3 + 0] = gr[0];
    b.gT64[(int64_t)p * 3 + 1] = gr[1];
    b.gT64[(int64_t)p * 3 + 2] = gr[2];
  } else {
    b.gT[(int64_t)p * 3 + 0] = (float)gr[0];
    b.gT[(int64_t)p * 3 + 1] = (float)gr[1];
    b.gT[(int64_t)p * 3 + 2] = (float)gr[2];
  }
}

// ---------------------------------------------------------------- residual

__global__ void k_residual(CatView cat, int C, int64_t n, const double* theta, int64_t theta_stride,
                           int whiten, BatchBufs b, int32_t* act) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)C * n) return;
  // T of each entry carries its event's origin time: T_i + t_i - (T_j + t_j)
  const TRec ti = b.tr[2 * q], tj = b.tr[2 * q + 1];  // both entries, one 32-byte read
  const double r = b.tau[q] - (ti.T - tj.T);
  if (b.r) b.r[q] = r;
  const double s2 = cat.sigma * cat.sigma;
  // S-phase scale; a catalog without S groups (L_p = L) never reads the group
  const double zs = cat.L_p < cat.L && b.sta[2 * q] >= cat.L_p ? cat.zscale_s : 1.0;
  const int32_t pi = ti.p, pj = tj.p;
  double z;
  if (whiten == kWhitenL1) {
    z = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);  // d|r|/dr, 0 at 0
  } else if (whiten == 0 || cat.kappa == 0.0) {
    z = r / s2 * zs;
  } else if (whiten == 1 || ((pi & pj) & kSingle)) {
    // diagonal whitening, or (exact) an edge alone in its two nodes: Sigma_B
    // restricted to it is sigma^2 + 2 kappa^2 w
    z = r / (s2 + 2.0 * cat.kappa * cat.kappa * b.w[q]) * zs;
  } else {
    WRec x;
    x.w = b.w[q];
    x.r = r;
    x.hi = ti.head;
    x.hj = tj.head;
    x.pad[0] = x.pad[1] = 0;
    b.wr[q] = x;
    act[x.hi] = 1;
    act[x.hj] = 1;
    return;  // z from the solve (k_tree_lds or k_tree_solve)
  }
  b.zp[pi & kPosMask] = z;  // the sign of each entry's term in the per-event sums
  b.zp[pj & kPosMask] = -z;
}

// ---------------------------------------------------------------- exact whitening
// Sigma_B = s2 I + k2 U U^T, U = W^{1/2} A_B.  z = (r - U y)/s2 with
// (lambda I + U^T U) y = U^T r, lambda = s2/k2.  U^T U is the w-weighted
// Laplacian of the batch's event graph in each group: one system per
// (chain, group).  The nodes taken here are those of the observations that
// share a node with another one (every neighbour of such a node is one too).

constexpr int32_t kActive = -1;
constexpr int32_t kCore = 1 << 30;  // solved by CG after the peeling rounds
constexpr int kListTB = 512;
constexpr int kListU = 4;  // positions per thread whose loads are in flight together

// The system lists: block (b, c) of the grid covers positions [2 n c + b span,
// ...) of chain c; pass 1 counts its marked nodes per group in LDS and writes
// the counts to sys[(c L + g) nb + b]; after the scan, pass 2 places each
// node in its system's list (slot from an LDS counter: the order within a
// list does not matter to the solver) and initialises it: the diagonal
// lambda + sum w and right-hand side (U^T r) = sum +-sqrt(w) r over its
// entries in CSR order, and per entry its record (weight, signed residual,
// the node at the other end).  hist: L ints of dynamic LDS.  Both passes
// take the block's positions kListU per thread at a time and issue each
// stage's loads for all of them before the first is used.
__global__ __launch_bounds__(kListTB) void k_list_count(int64_t n, int L, int64_t nb, int64_t span,
                                                       BatchBufs b, SolveBufs sv) {
  extern __shared__ int32_t hist[];
  const int64_t c = blockIdx.y, bk = blockIdx.x;
  for (int g = threadIdx.x; g < L; g += kListTB) hist[g] = 0;
  __syncthreads();
  const int64_t p0 = 2 * n * c + bk * span;
  const int64_t p1 = min(2 * n * (c + 1), p0 + span);
  for (int64_t base = p0 + threadIdx.x; base < p1; base += (int64_t)kListTB * kListU) {
    int32_t on[kListU], g[kListU];
#pragma unroll
    for (int u = 0; u < kListU; ++u) {
      const int64_t p = base + u * kListTB;
      on[u] = p < p1 ? sv.act[p] : 0;
    }
#pragma unroll
    for (int u = 0; u < kListU; ++u)
      if (on[u]) g[u] = b.pgr[base + u * kListTB];
#pragma unroll
    for (int u = 0; u < kListU; ++u)
      if (on[u]) atomicAdd(&hist[g[u]], 1);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < L; g += kListTB) sv.sys[(c * L + g) * nb + bk] = hist[g];
  if (c == 0 && bk == 0 && threadIdx.x == 0) sv.sys[(int64_t)gridDim.y * L * nb] = 0;
}

__global__ __launch_bounds__(kListTB) void k_list_fill(int64_t n, int L, int64_t nb, int64_t span,
                                                      double lambda, int64_t E, BatchBufs b,
                                                      SolveBufs sv) {
  extern __shared__ int32_t hist[];
  const int64_t c = blockIdx.y, bk = blockIdx.x;
  for (int g = threadIdx.x; g < L; g += kListTB) hist[g] = 0;
  __syncthreads();
  const int64_t p0 = 2 * n * c + bk * span;
  const int64_t p1 = min(2 * n * (c + 1), p0 + span);
  for (int64_t base = p0 + threadIdx.x; base < p1; base += (int64_t)kListTB * kListU) {
    // the flags; then group, end and first entry of each marked node; then
    // that entry's record (weight, residual, both nodes)
    int32_t on[kListU], g[kListU], pe[kListU], e0[kListU];
    WRec x0[kListU];
#pragma unroll
    for (int u = 0; u < kListU; ++u) {
      const int64_t p = base + u * kListTB;
      on[u] = p < p1 ? sv.act[p] : 0;
    }
#pragma unroll
    for (int u = 0; u < kListU; ++u) {
      if (!on[u]) continue;
      const int64_t p = base + u * kListTB;
      g[u] = b.pgr[p];
      pe[u] = b.nend[p];
      e0[u] = b.csr[p];
    }
#pragma unroll
    for (int u = 0; u < kListU; ++u)
      if (on[u]) x0[u] = b.wr[e0[u] >> 1];
#pragma unroll
    for (int u = 0; u < kListU; ++u) {
      if (!on[u]) continue;
      const int32_t p = (int32_t)(base + u * kListTB);
      const int32_t slot = atomicAdd(&hist[g[u]], 1);
      const int32_t at = sv.sys[(c * L + g[u]) * nb + bk] + slot;
      sv.list[at] = p;
      sv.lidx[p] = at - sv.sys[(c * L + g[u]) * nb];
      double A = lambda, rhs = 0.0;
      for (int32_t f = p; f < pe[u]; ++f) {
        const int32_t e = f == p ? e0[u] : b.csr[f];
        const WRec x = f == p ? x0[u] : b.wr[e >> 1];
        A += x.w;
        rhs += ((e & 1) ? -1.0 : 1.0) * sqrt(x.w) * x.r;
        ERec en;
        en.w = x.w;
        en.rs = (e & 1) ? -x.r : x.r;
        en.nbr = (e & 1) ? x.hi : x.hj;  // the node at the other end
        en.pad = 0;
        sv.ent[f] = en;
      }
      NodeRec nr;
      nr.A = A;
      nr.b = rhs;
      nr.q = p;
      nr.ne = pe[u] - p;
      sv.nrec[at] = nr;  // list order: the LDS solver reads its system in one stream
    }
  }
}

struct SolveArgs {
  const int32_t* nend;  // entries of node q: CSR positions [q, nend[q])
  const ERec* ent;      // per position: weight, signed residual, node at the other end
  const int32_t* sys;   // list offsets: system s starts at sys[s nb]
  int64_t nb;
  int32_t* list;        // nodes of each system (first positions)
  double* A;            // diagonal, Schur-updated as leaves are eliminated
  double* b;            // right-hand side, Schur-updated
  double* y;            // solution
  double* Wp;           // weight to the parent at elimination
  double* rr;           // CG vectors for the nodes left on cycles
  double* p;
  double* ap;
  int32_t* state;       // kActive, kCore, or the round in which the node was removed
  int32_t* nstate;
  int32_t* par;         // parent of an eliminated node (-1: solved on its own)
  int32_t* next;        // scratch: the next round's list (same offsets as list)
  int32_t* elim;        // scratch: the elimination order (same offsets as list)
  double lambda;
  int max_rounds;
  int max_iter;
  double tol2;     // CG stops once |res|^2 <= tol2 |rhs|^2
  double accept2;  // after its passes, |res|^2 > accept2 |rhs|^2 raises kErrSolve
  int* err;        // error bits of the step
  const int32_t* lidx;  // index of a node in its system's list (at its first position)
  const NodeRec* nrec;  // the nodes in list order
  int32_t* spill;       // per system: 1 if k_tree_solve takes it
  int lds_off;          // 1: every system to k_tree_solve (SPIDER_TREE_GLOBAL, for tests)
  double* zp;           // per position: the whitened residual, negated at the second entry
  double sigma;         // sigma of the catalog's P groups
  double zscale_s;      // z scale of S groups (system s has group s mod L)
  int L, L_p;
};

// The whitened residual z = (r - sqrt(w) (y_i - y_j)) / sigma^2 (times the
// group's scale) at one entry of an observation, negated at its second
// entry: with rs and the two y taken from that entry's side (rs = -r and
// the node's own y first at the second entry) the value is exactly -z,
// since every step of the expression is odd in (rs, y_own - y_other).
__device__ __forceinline__ double signed_z(double rs, double w, double y_own, double y_other,
                                           double sigma, double zs) {
  return (rs - sqrt(w) * (y_own - y_other)) / (sigma * sigma) * zs;
}

constexpr int kMaxRounds = 64;
constexpr int kWaveCore = 64;  // cores up to this size: CG in one wave
constexpr int kWaveNb = 8;     // core entries per node held for the one-wave CG
constexpr int kTreeBlock = 1024;  // threads per (chain, group) system
constexpr int kCoreLds = 4096;    // cores up to this size are sorted in LDS

// Appends, in order, the n items item(k) that satisfy keep(k) to out: thread
// t handles the contiguous items [t per, (t + 1) per), an exclusive scan of
// the per-thread counts over the block (butterfly within waves, then the wave
// totals) gives each thread its first output slot.  Returns the number
// appended.  All threads of the block call it; scan holds TB / 64 ints.
template <int TB, class Keep, class Item, class Out>
__device__ int32_t block_compact(int32_t n, Keep&& keep, Item&& item, Out* out, int32_t* scan) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int32_t per = (n + TB - 1) / TB;
  const int32_t k0 = t * per, k1 = min(n, k0 + per);
  int32_t cnt = 0;
  for (int32_t k = k0; k < k1; ++k) cnt += keep(k) ? 1 : 0;
  int32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t x = __shfl_up(incl, d, 64);
    if (lane >= d) incl += x;
  }
  if (lane == 63) scan[w] = incl;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int v = 0; v < TB / 64; ++v) {
    const int32_t x = scan[v];
    if (v < w) before += x;
    total += x;
  }
  int32_t o = before + incl - cnt;
  for (int32_t k = k0; k < k1; ++k)
    if (keep(k)) out[o++] = item(k);
  __syncthreads();
  return total;
}

// One workgroup per (chain, group) system of (lambda I + L) y = U^T r over
// its listed nodes (the list's order is arbitrary; nothing below depends on
// it except the CG sums, which run over the core sorted by node):
//  1. Peel leaves in rounds: a node whose active neighbours are all one node
//     p (possibly over several parallel edges of total weight W) is
//     eliminated into p (Schur complement: A_p -= W^2/A_q, b_p += W b_q/A_q);
//     of two nodes that are each other's only neighbour the larger one is
//     eliminated; a node with no active neighbour is solved, y = b/A.
//     Parents gather their leaves' updates in entry order (deterministic).
//  2. Nodes left on cycles after the rounds: Jacobi-preconditioned CG on
//     the Schur-complemented system of those nodes only.
//  3. Back substitution in reverse round order: y_q = (b_q + W y_p)/A_q.
// Exact up to FP64 rounding for forests; the minibatch graphs are forests
// of small trees apart from rare cycles.
// Jacobi-CG on a core of n <= 64 nodes in one wave (the workgroup's first):
// lane k holds the k-th smallest node and its core entries (lane of the other
// end, weight) in its own LDS row; the neighbours' values are shuffles and the
// sums xor butterflies (the same bits in every lane), so an iteration costs no
// barrier and no memory round trip.  The same passes, tolerances and error
// bit as the workgroup CG.  Returns false, having written nothing, when a
// node has more than kWaveNb core entries.
__device__ bool wave_core_cg(const SolveArgs& a, const int32_t* core, int32_t n,
                             int32_t (*nb_sh)[kWaveNb], double (*w_sh)[kWaveNb]) {
  const int lane = threadIdx.x & 63;
  const bool on = lane < n;
  const int32_t mine = on ? core[lane] : INT32_MAX;
  int rank = 0;
  for (int i = 0; i < n; ++i) rank += __shfl(mine, i, 64) < mine ? 1 : 0;
  int32_t q = INT32_MAX;
  for (int i = 0; i < n; ++i) {
    const int ri = __shfl(rank, i, 64);
    const int32_t vi = __shfl(mine, i, 64);
    if (ri == lane) q = vi;
  }
  int cnt = 0;
  bool over = false;
  if (on) {
    const int32_t e1 = a.nend[q];
    for (int32_t e = q; e < e1; ++e) {
      const int32_t pn = a.ent[e].nbr;
      if (a.state[pn] != kActive) continue;
      if (cnt == kWaveNb) {
        over = true;
        break;
      }
      nb_sh[lane][cnt] = pn;
      w_sh[lane][cnt] = a.ent[e].w;
      ++cnt;
    }
  }
  if (__any(over)) return false;
  int maxc = cnt;
  for (int m = 32; m > 0; m >>= 1) maxc = max(maxc, __shfl_xor(maxc, m, 64));
  // entries' other ends as lanes: lower bound in the sorted nodes (a
  // wave-uniform number of steps, so every lane takes part in each shuffle)
  for (int s = 0; s < maxc; ++s) {
    const int32_t target = s < cnt ? nb_sh[lane][s] : INT32_MAX;
    int pos = 0;
    for (int step = 32; step >= 1; step >>= 1) {
      const int cand = pos + step;
      const int32_t v = __shfl(q, (cand - 1) & 63, 64);
      if (cand <= n && v < target) pos = cand;
    }
    if (s < cnt) nb_sh[lane][s] = pos;
  }
  auto wsum = [](double v) {
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
  };
  const double Aq = on ? a.A[q] : 1.0;
  const double bq = on ? a.b[q] : 0.0;
  double y = 0.0, rr = 0.0, p = 0.0;
  const double bb = wsum(bq * bq);
  double rn = bb;
  for (int pass = 0; pass < 3 && bb > 0.0; ++pass) {
    // the true residual b - A y of the current y
    double v = bq - Aq * y;
    for (int s = 0; s < maxc; ++s) {
      const double yv = __shfl(y, s < cnt ? nb_sh[lane][s] : lane, 64);
      if (s < cnt) v += w_sh[lane][s] * yv;
    }
    rr = on ? v : 0.0;
    p = rr / Aq;
    rn = wsum(rr * rr);
    double rz = wsum(rr * rr / Aq);
    if (rn <= a.tol2 * bb) break;
    for (int it = 0; it < a.max_iter; ++it) {
      double ap = Aq * p;
      for (int s = 0; s < maxc; ++s) {
        const double pv = __shfl(p, s < cnt ? nb_sh[lane][s] : lane, 64);
        if (s < cnt) ap -= w_sh[lane][s] * pv;
      }
      if (!on) ap = 0.0;
      const double pap = wsum(p * ap);
      const double alpha = rz / pap;
      y += alpha * p;
      rr -= alpha * ap;
      rn = wsum(rr * rr);
      const double rz_new = wsum(rr * rr / Aq);
      if (rn <= a.tol2 * bb) break;
      const double beta = rz_new / rz;
      rz = rz_new;
      p = rr / Aq + beta * p;
    }
  }
  if (lane == 0 && bb > 0.0 && !(rn <= a.accept2 * bb)) atomicOr(a.err, kErrSolve);
  if (on) {
    a.y[q] = y;
    a.state[q] = kCore;
  }
  return true;
}

// The one-wave core CG of k_tree_lds: nodes are indices into the system's
// list (positions gpos), entries in LDS (eoff, snb), state sst; y replaces b
// in sB.  Same ordering (by CSR position), arithmetic and tolerances as
// wave_core_cg.
template <class Q>
__device__ bool wave_core_cg_lds(const SolveArgs& a, const uint16_t* core, int32_t n,
                                 Q&& gpos, const uint16_t* eoff, const uint16_t* snb,
                                 uint8_t* sst, const double* sA, double* sB,
                                 double (*w_sh)[kWaveNb], int32_t (*nb_sh)[kWaveNb]) {
  constexpr uint8_t kActiveL = 255, kCoreL = 254;
  const int lane = threadIdx.x & 63;
  const bool on = lane < n;
  const int32_t mine_i = on ? core[lane] : 0;
  const int32_t mine = on ? gpos(mine_i) : INT32_MAX;
  int rank = 0;
  for (int k = 0; k < n; ++k) rank += __shfl(mine, k, 64) < mine ? 1 : 0;
  int32_t node = 0, key = INT32_MAX;  // this lane's node (list index) and position
  for (int k = 0; k < n; ++k) {
    const int rk = __shfl(rank, k, 64);
    const int32_t ik = __shfl(mine_i, k, 64);
    const int32_t vk = __shfl(mine, k, 64);
    if (rk == lane) {
      node = ik;
      key = vk;
    }
  }
  int cnt = 0;
  bool over = false;
  if (on) {
    const int32_t e0 = eoff[node], e1 = eoff[node + 1];
    for (int32_t x = e0; x < e1; ++x) {
      const int32_t pn = snb[x];
      if (sst[pn] != kActiveL) continue;
      if (cnt == kWaveNb) {
        over = true;
        break;
      }
      nb_sh[lane][cnt] = gpos(pn);
      w_sh[lane][cnt] = a.ent[key + (x - e0)].w;
      ++cnt;
    }
  }
  if (__any(over)) return false;
  int maxc = cnt;
  for (int m = 32; m > 0; m >>= 1) maxc = max(maxc, __shfl_xor(maxc, m, 64));
  for (int s = 0; s < maxc; ++s) {
    const int32_t target = s < cnt ? nb_sh[lane][s] : INT32_MAX;
    int pos = 0;
    for (int step = 32; step >= 1; step >>= 1) {
      const int cand = pos + step;
      const int32_t v = __shfl(key, (cand - 1) & 63, 64);
      if (cand <= n && v < target) pos = cand;
    }
    if (s < cnt) nb_sh[lane][s] = pos;
  }
  auto wsum = [](double v) {
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
  };
  const double Aq = on ? sA[node] : 1.0;
  const double bq = on ? sB[node] : 0.0;
  double y = 0.0, rr = 0.0, p = 0.0;
  const double bb = wsum(bq * bq);
  double rn = bb;
  for (int pass = 0; pass < 3 && bb > 0.0; ++pass) {
    double v = bq - Aq * y;
    for (int s = 0; s < maxc; ++s) {
      const double yv = __shfl(y, s < cnt ? nb_sh[lane][s] : lane, 64);
      if (s < cnt) v += w_sh[lane][s] * yv;
    }
    rr = on ? v : 0.0;
    p = rr / Aq;
    rn = wsum(rr * rr);
    double rz = wsum(rr * rr / Aq);
    if (rn <= a.tol2 * bb) break;
    for (int it = 0; it < a.max_iter; ++it) {
      double ap = Aq * p;
      for (int s = 0; s < maxc; ++s) {
        const double pv = __shfl(p, s < cnt ? nb_sh[lane][s] : lane, 64);
        if (s < cnt) ap -= w_sh[lane][s] * pv;
      }
      if (!on) ap = 0.0;
      const double pap = wsum(p * ap);
      const double alpha = rz / pap;
      y += alpha * p;
      rr -= alpha * ap;
      rn = wsum(rr * rr);
      const double rz_new = wsum(rr * rr / Aq);
      if (rn <= a.tol2 * bb) break;
      const double beta = rz_new / rz;
      rz = rz_new;
      p = rr / Aq + beta * p;
    }
  }
  if (lane == 0 && bb > 0.0 && !(rn <= a.accept2 * bb)) atomicOr(a.err, kErrSolve);
  if (on) {
    sB[node] = y;
    sst[node] = kCoreL;
  }
  return true;
}

template <int TB>
__global__ __launch_bounds__(TB) void k_tree_solve(SolveArgs a) {
  __shared__ double sh[TB / 64];
  __shared__ int32_t warp_base[TB / 64];
  __shared__ int32_t elim_start[kMaxRounds + 2];
  __shared__ int32_t core_sh[kCoreLds];
  __shared__ int32_t wc_nb[kWaveCore][kWaveNb];
  __shared__ double wc_w[kWaveCore][kWaveNb];
  __shared__ int wc_done;
  if (!a.spill[blockIdx.x]) return;  // solved in LDS by k_tree_lds
  const int32_t off = a.sys[blockIdx.x * a.nb];
  int32_t nl = a.sys[(blockIdx.x + 1) * a.nb] - off;
  if (nl <= 0) return;
  const int t = threadIdx.x;
  // the system's nodes at their first positions: A, b, active, no parent
  for (int32_t k = t; k < nl; k += TB) {
    const NodeRec nr = a.nrec[off + k];
    a.A[nr.q] = nr.A;
    a.b[nr.q] = nr.b;
    a.state[nr.q] = kActive;
    a.par[nr.q] = -1;
  }
  __syncthreads();
  int32_t* act = a.list + off;
  int32_t* act_next = a.next + off;
  int32_t* elim = a.elim + off;
  int32_t n_elim = 0;

  // ---- 1. peeling rounds over the active nodes
  int rounds = 0;
  for (; rounds < a.max_rounds && nl > 0; ++rounds) {
    if (t == 0) elim_start[rounds] = n_elim;
    int changed = 0;
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t q = act[k];
      int32_t p0 = -1;
      double W = 0.0;
      bool multi = false;
      for (int32_t e = q; e < a.nend[q]; ++e) {
        const int32_t pn = a.ent[e].nbr;
        if (a.state[pn] != kActive) continue;
        if (p0 < 0) {
          p0 = pn;
          W = a.ent[e].w;
        } else if (pn == p0) {
          W += a.ent[e].w;
        } else {
          multi = true;
          break;
        }
      }
      int32_t ns = kActive;
      if (p0 < 0) {
        ns = rounds;  // isolated: solved directly
        a.par[q] = -1;
      } else if (!multi) {
        bool p0_other = false;
        for (int32_t e = p0; e < a.nend[p0]; ++e) {
          const int32_t pn = a.ent[e].nbr;
          if (pn != q && a.state[pn] == kActive) {
            p0_other = true;
            break;
          }
        }
        if (p0_other || q > p0) {
          ns = rounds;
          a.par[q] = p0;
          a.Wp[q] = W;
        }
      }
      a.nstate[q] = ns;
      changed |= (ns != kActive);
    }
    changed = __syncthreads_or(changed);
    if (!changed) break;
    // parents gather the Schur updates of this round's leaves
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t q = act[k];
      if (a.nstate[q] == kActive) {
        const int32_t e0 = q, e1 = a.nend[q];
        double dA = 0.0, db = 0.0;
        for (int32_t e = e0; e < e1; ++e) {
          const int32_t pn = a.ent[e].nbr;
          if (a.nstate[pn] != rounds || a.par[pn] != q) continue;
          bool first = true;
          for (int32_t f = e0; f < e; ++f)
            if (a.ent[f].nbr == pn) {
              first = false;
              break;
            }
          if (!first) continue;
          const double Ap = a.A[pn], Wn = a.Wp[pn];
          dA += Wn * Wn / Ap;
          db += Wn * a.b[pn] / Ap;
        }
        a.A[q] -= dA;
        a.b[q] += db;
      }
    }
    __syncthreads();
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t q = act[k];
      a.state[q] = a.nstate[q];
    }
    __syncthreads();
    n_elim += block_compact<TB>(
        nl, [&](int32_t k) { return a.state[act[k]] != kActive; }, [&](int32_t k) { return act[k]; },
        elim + n_elim, warp_base);
    nl = block_compact<TB>(
        nl, [&](int32_t k) { return a.state[act[k]] == kActive; }, [&](int32_t k) { return act[k]; },
        act_next, warp_base);
    int32_t* tmp = act;
    act = act_next;
    act_next = tmp;
  }
  if (t == 0) elim_start[rounds] = n_elim;
  __syncthreads();

  // ---- 2. nodes still active sit on cycles (or on paths longer than the
  // round cap): CG on them only, over the core sorted by node (the sums then
  // run in a fixed order).  Each pass starts from the true residual b - A y
  // of the current y (the first from y = 0), so later passes correct the
  // drift of CG's recursively updated residual.
  int32_t* core = act;
  const int32_t ncore = nl;
  bool core_done = false;
  if (ncore > 0 && ncore <= kWaveCore) {
    if (t < 64) {
      const bool ok = wave_core_cg(a, core, ncore, wc_nb, wc_w);
      if (t == 0) wc_done = ok ? 1 : 0;
    }
    __syncthreads();
    core_done = wc_done != 0;
  }
  if (ncore > 0 && !core_done) {
    if (ncore <= kCoreLds) {
      for (int32_t k = t; k < ncore; k += TB) core_sh[k] = core[k];
      __syncthreads();
      block_sort_any(ncore, [&](int32_t i) { return (uint64_t)(uint32_t)core_sh[i]; },
                     [&](int32_t i, uint64_t x) { core_sh[i] = (int32_t)x; });
      for (int32_t k = t; k < ncore; k += TB) core[k] = core_sh[k];
    } else {
      block_sort_any(ncore, [&](int32_t i) { return (uint64_t)(uint32_t)core[i]; },
                     [&](int32_t i, uint64_t x) { core[i] = (int32_t)x; });
    }
    __syncthreads();
    double bb = 0.0;
    for (int32_t k = t; k < ncore; k += TB) {
      const int32_t q = core[k];
      a.y[q] = 0.0;
      bb += a.b[q] * a.b[q];
    }
    bb = block_sum<TB>(bb, sh);
    double rn = bb;
    for (int pass = 0; pass < 3 && bb > 0.0; ++pass) {
      double rz = 0.0;
      rn = 0.0;
      for (int32_t k = t; k < ncore; k += TB) {
        const int32_t q = core[k];
        double v = a.b[q] - a.A[q] * a.y[q];
        for (int32_t e = q; e < a.nend[q]; ++e) {
          const int32_t pn = a.ent[e].nbr;
          if (a.state[pn] == kActive) v += a.ent[e].w * a.y[pn];
        }
        a.rr[q] = v;
        a.p[q] = v / a.A[q];
        rn += v * v;
        rz += v * v / a.A[q];
      }
      rn = block_sum<TB>(rn, sh);
      rz = block_sum<TB>(rz, sh);
      if (rn <= a.tol2 * bb) break;
      for (int it = 0; it < a.max_iter; ++it) {
        double pap = 0.0;
        for (int32_t k = t; k < ncore; k += TB) {
          const int32_t q = core[k];
          double v = a.A[q] * a.p[q];
          for (int32_t e = q; e < a.nend[q]; ++e) {
            const int32_t pn = a.ent[e].nbr;
            if (a.state[pn] == kActive) v -= a.ent[e].w * a.p[pn];
          }
          a.ap[q] = v;
          pap += a.p[q] * v;
        }
        pap = block_sum<TB>(pap, sh);
        const double alpha = rz / pap;
        double rz_new = 0.0;
        rn = 0.0;
        for (int32_t k = t; k < ncore; k += TB) {
          const int32_t q = core[k];
          a.y[q] += alpha * a.p[q];
          const double rq = a.rr[q] - alpha * a.ap[q];
          a.rr[q] = rq;
          rn += rq * rq;
          rz_new += rq * rq / a.A[q];
        }
        rn = block_sum<TB>(rn, sh);
        rz_new = block_sum<TB>(rz_new, sh);
        if (rn <= a.tol2 * bb) break;
        const double beta = rz_new / rz;
        rz = rz_new;
        for (int32_t k = t; k < ncore; k += TB) {
          const int32_t q = core[k];
          a.p[q] = a.rr[q] / a.A[q] + beta * a.p[q];
        }
        __syncthreads();
      }
    }
    if (t == 0 && bb > 0.0 && !(rn <= a.accept2 * bb)) atomicOr(a.err, kErrSolve);
    for (int32_t k = t; k < ncore; k += TB) a.state[core[k]] = kCore;
    __syncthreads();
  }

  // ---- 3. back substitution in reverse elimination order, one round at a time
  for (int rnd = rounds - 1; rnd >= 0; --rnd) {
    for (int32_t k = elim_start[rnd] + t; k < elim_start[rnd + 1]; k += TB) {
      const int32_t q = elim[k];
      const int32_t pn = a.par[q];
      a.y[q] = pn < 0 ? a.b[q] / a.A[q] : (a.b[q] + a.Wp[q] * a.y[pn]) / a.A[q];
    }
    __syncthreads();
  }
  // z at every entry of the system's nodes (y at the nodes' first positions)
  const int32_t n_sys = a.sys[(blockIdx.x + 1) * a.nb] - off;
  const int g = (int)(blockIdx.x % a.L);
  const double zs = g >= a.L_p ? a.zscale_s : 1.0;
  for (int32_t k = t; k < n_sys; k += TB) {
    const NodeRec nr = a.nrec[off + k];
    const double yq = a.y[nr.q];
    for (int32_t x = 0; x < nr.ne; ++x) {
      const int32_t f = nr.q + x;
      const ERec en = a.ent[f];
      a.zp[f] = signed_z(en.rs, en.w, yq, a.y[en.nbr], a.sigma, zs);
    }
  }
}

__global__ void k_obs_z(int64_t Q, BatchBufs b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  b.z[q] = b.zp[b.tr[2 * q].p & kPosMask];  // the first entry carries +z
}

// ---------------------------------------------------------------- reduce

// Per-event gradient sums over the CSR segments, read position by position
// (coalesced).  Pass A: each wave takes 64 consecutive positions, forms
// v = scale z (dT/dx, 1) per position (z carries the entry's sign) and runs
// a segmented inclusive scan over its lanes (a fixed order of DPP steps:
// within 16-lane rows, then across rows); a segment that starts and ends
// inside the wave is written
// to G at its last lane, the wave's first and last segment sums go to
// part[w] = {head, tail} when they reach past the wave.  Pass B: every key
// whose segment spans waves sums tail(first wave) + head(next waves) in wave
// order; empty keys get 0.  Every sum has a fixed order.
constexpr int kReduceTB = 256;

// Lane movement by DPP (no LDS): row_shr:D within each 16-lane row, and the
// broadcasts of lane 15 of rows 0 and 2 into rows 1 and 3 (row_bcast:15) and
// of lane 31 into rows 2 and 3 (row_bcast:31).  Lanes without a source, and
// rows outside the mask, read 0.
constexpr int kDppRowShr = 0x110, kDppBcast15 = 0x142, kDppBcast31 = 0x143;

template <int Ctrl, int RowMask>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, Ctrl, RowMask, 0xF, true);
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 x = __builtin_bit_cast(int2, v);
  int2 y;
  y.x = dpp_i32<Ctrl, RowMask>(x.x);
  y.y = dpp_i32<Ctrl, RowMask>(x.y);
  return __builtin_bit_cast(double, y);
}

// One step of the segmented inclusive scan of four sums: each lane adds the
// sums held at its DPP source when ok (the source lies in the lane's
// segment), in the order source + own.
template <int Ctrl, int RowMask>
__device__ __forceinline__ void seg_step(bool ok, double& v0, double& v1, double& v2, double& v3) {
  const double y0 = dpp_f64<Ctrl, RowMask>(v0), y1 = dpp_f64<Ctrl, RowMask>(v1);
  const double y2 = dpp_f64<Ctrl, RowMask>(v2), y3 = dpp_f64<Ctrl, RowMask>(v3);
  if (ok) {
    v0 = y0 + v0;
    v1 = y1 + v1;
    v2 = y2 + v2;
    v3 = y3 + v3;
  }
}

__global__ __launch_bounds__(kReduceTB) void k_reduce_waves(int64_t E, int64_t n, int M,
                                                           double scale, BatchBufs b, double* G,
                                                           double4* part) {
  const int64_t p = (int64_t)blockIdx.x * kReduceTB + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t w = p >> 6, wave0 = w << 6;
  // keys are >= 0; outside [0, E) the sentinels -1 (before) and -2 (after),
  // -3 for a lane past the end (positions fit in 32 bits: 32-bit division)
  const uint32_t span = (uint32_t)(2 * n);
  auto key_of = [&](int64_t q) -> int64_t {
    return q < 0 ? -1 : q >= E ? -2 : (int64_t)((uint32_t)q / span) * M + b.pev[q];
  };
  const bool valid = p < E;
  const int64_t key = valid ? key_of(p) : -3;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  if (valid) {
    const double cz = scale * b.zp[p];  // zp is negated at an observation's second entry
    const float* g = b.gT + p * 3;
    v0 = cz * (double)g[0];
    v1 = cz * (double)g[1];
    v2 = cz * (double)g[2];
    v3 = cz;
  }
  const int64_t prev = __shfl_up(key, 1, 64), next = __shfl_down(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const bool tail = lane == 63 || next != key;
  // lane of this lane's segment head within the wave (inclusive max scan)
  int hl = head ? lane : 0;
  hl = max(hl, dpp_i32<kDppRowShr + 1, 0xF>(hl));
  hl = max(hl, dpp_i32<kDppRowShr + 2, 0xF>(hl));
  hl = max(hl, dpp_i32<kDppRowShr + 4, 0xF>(hl));
  hl = max(hl, dpp_i32<kDppRowShr + 8, 0xF>(hl));
  hl = max(hl, dpp_i32<kDppBcast15, 0xA>(hl));
  hl = max(hl, dpp_i32<kDppBcast31, 0xC>(hl));
  // the segmented scan: within each row, then across rows
  const int r = lane & 15, row0 = lane & 48;
  seg_step<kDppRowShr + 1, 0xF>(r >= 1 && lane - 1 >= hl, v0, v1, v2, v3);
  seg_step<kDppRowShr + 2, 0xF>(r >= 2 && lane - 2 >= hl, v0, v1, v2, v3);
  seg_step<kDppRowShr + 4, 0xF>(r >= 4 && lane - 4 >= hl, v0, v1, v2, v3);
  seg_step<kDppRowShr + 8, 0xF>(r >= 8 && lane - 8 >= hl, v0, v1, v2, v3);
  seg_step<kDppBcast15, 0xA>((row0 == 16 || row0 == 48) && hl < row0, v0, v1, v2, v3);
  seg_step<kDppBcast31, 0xC>(row0 >= 32 && hl < 32, v0, v1, v2, v3);
  if (!valid || !tail) return;
  // does the segment reach past the wave's first or last position?
  const bool open_left = hl == 0 && key_of(wave0 - 1) == key;
  const bool open_right = lane == 63 && key_of(p + 1) == key;
  if (!open_left && !open_right) {
    *(double4*)(G + key * 4) = make_double4(v0, v1, v2, v3);
    return;
  }
  if (open_left) part[2 * w] = make_double4(v0, v1, v2, v3);       // head of the wave
  if (open_right) part[2 * w + 1] = make_double4(v0, v1, v2, v3);  // tail of the wave
}

__global__ void k_reduce_keys(int64_t K, BatchBufs b, double* G, const double4* part) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int64_t p0 = b.start[k], p1 = b.start[k + 1];
  if (p1 == p0) {
    *(double4*)(G + k * 4) = make_double4(0.0, 0.0, 0.0, 0.0);
    return;
  }
  const int64_t w0 = p0 >> 6, w1 = (p1 - 1) >> 6;
  if (w0 == w1) return;  // written by k_reduce_waves
  double4 s = part[2 * w0 + 1];
  for (int64_t w = w0 + 1; w <= w1; ++w) {
    const double4 h = part[2 * w];
    s.x += h.x;
    s.y += h.y;
    s.z += h.z;
    s.w += h.w;
  }
  *(double4*)(G + k * 4) = s;
}

// ---------------------------------------------------------------- per-slot outputs

__global__ void k_batch_terms_out(int64_t n, BatchBufs b, const double* theta, double* Ti,
                                  double* Tj, double* gi, double* gj, double* r, double* z) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  // tr holds T + t of each entry
  const TRec ti = b.tr[2 * q], tj = b.tr[2 * q + 1];
  if (Ti) Ti[q] = ti.T - theta[(int64_t)b.ev[2 * q] * 4 + 3];
  if (Tj) Tj[q] = tj.T - theta[(int64_t)b.ev[2 * q + 1] * 4 + 3];
  const int64_t pi = ti.p & kPosMask, pj = tj.p & kPosMask;
  for (int a = 0; a < 3; ++a) {
    if (gi) gi[q * 3 + a] = b.gT64[pi * 3 + a];
    if (gj) gj[q * 3 + a] = b.gT64[pj * 3 + a];
  }
  if (r) r[q] = b.r[q];
  if (z) z[q] = b.zp[pi];  // the first entry carries +z
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

// Linear-regime test of the n slots of one chain's batch (entries 2q, 2q + 1
// = events i, j): dT = T_j - T_i, lin = grad T(x_i) . (x_j - x_i), keep[q] =
// |dT - lin| <= e_max |dT|; the kept count is added to *count.
__global__ void k_linear_keep(const BatchBufs b, const double* theta, int64_t n, double e_max,
                              uint8_t* keep, unsigned long long* count) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned int k = 0;
  if (q < n) {
    const double* xi = theta + (int64_t)b.ev[2 * q] * 4;
    const double* xj = theta + (int64_t)b.ev[2 * q + 1] * 4;
    const double* g = b.gT64 + (int64_t)(b.tr[2 * q].p & kPosMask) * 3;
    // tr holds T + t of each entry
    const double dT = (b.tr[2 * q + 1].T - xj[3]) - (b.tr[2 * q].T - xi[3]);
    const double lin = g[0] * (xj[0] - xi[0]) + g[1] * (xj[1] - xi[1]) + g[2] * (xj[2] - xi[2]);
    k = fabs(dT - lin) <= e_max * fabs(dT) ? 1u : 0u;
    keep[q] = (uint8_t)k;
  }
  block_count_add(k, count);
}

// The block CG of k_tree_solve for a cycle core of 65..TB nodes held in LDS,
// with the same arithmetic: one core node per thread in position order, the
// same sums in the same order (each node's core entries in entry order, then
// block_sum), y of the core in sB (b kept in a register) and p in sP.  Each
// node's core entries (at most kWaveNb, else false) and their weights are
// kept in registers.  order: n uint16 of scratch; cpos: TB ints of scratch;
// red: TB / 64 doubles.
template <int TB, class Q>
__device__ bool block_core_cg_lds(const SolveArgs& a, const uint16_t* core, int32_t n, Q&& gpos,
                                  const uint16_t* eoff, const uint16_t* snb, uint8_t* sst,
                                  const double* sA, double* sB, double* sP, uint16_t* order,
                                  int32_t* cpos, double* red) {
  constexpr uint8_t kActiveB = 255, kCoreB = 254;  // the LDS solver's node states
  const int t = threadIdx.x;
  const bool on = t < n;
  if (on) cpos[t] = gpos(core[t]);
  __syncthreads();
  if (on) {
    const int32_t mine = cpos[t];
    int32_t rank = 0;
    for (int32_t k = 0; k < n; ++k) rank += cpos[k] < mine ? 1 : 0;
    order[rank] = core[t];
  }
  __syncthreads();
  const int32_t node = on ? order[t] : 0;
  int32_t nbv[kWaveNb];
  double wv[kWaveNb];
  int over = 0;
  {
    const int32_t e0 = on ? eoff[node] : 0, e1 = on ? eoff[node + 1] : 0;
    const int32_t q = on ? gpos(node) : 0;
    int32_t x = e0;
#pragma unroll
    for (int k = 0; k < kWaveNb; ++k) {
      while (x < e1 && sst[snb[x]] != kActiveB) ++x;
      nbv[k] = -1;
      wv[k] = 0.0;
      if (x < e1) {
        nbv[k] = snb[x];
        wv[k] = a.ent[q + (x - e0)].w;
        ++x;
      }
    }
    while (x < e1 && sst[snb[x]] != kActiveB) ++x;
    over = x < e1 ? 1 : 0;
  }
  if (__syncthreads_or(over)) return false;
  const double Aq = on ? sA[node] : 1.0;
  const double bq = on ? sB[node] : 0.0;
  __syncthreads();
  if (on) sB[node] = 0.0;  // y = 0
  double bb = 0.0;
  if (on) bb += bq * bq;
  bb = block_sum<TB>(bb, red);
  double rn = bb, rr = 0.0, ap = 0.0;
  for (int pass = 0; pass < 3 && bb > 0.0; ++pass) {
    double rz = 0.0;
    rn = 0.0;
    if (on) {
      double v = bq - Aq * sB[node];
#pragma unroll
      for (int k = 0; k < kWaveNb; ++k)
        if (nbv[k] >= 0) v += wv[k] * sB[nbv[k]];
      rr = v;
      sP[node] = v / Aq;
      rn += v * v;
      rz += v * v / Aq;
    }
    rn = block_sum<TB>(rn, red);
    rz = block_sum<TB>(rz, red);
    if (rn <= a.tol2 * bb) break;
    for (int it = 0; it < a.max_iter; ++it) {
      double pap = 0.0;
      if (on) {
        double v = Aq * sP[node];
#pragma unroll
        for (int k = 0; k < kWaveNb; ++k)
          if (nbv[k] >= 0) v -= wv[k] * sP[nbv[k]];
        ap = v;
        pap += sP[node] * v;
      }
      pap = block_sum<TB>(pap, red);
      const double alpha = rz / pap;
      double rz_new = 0.0;
      rn = 0.0;
      if (on) {
        sB[node] += alpha * sP[node];
        const double rq = rr - alpha * ap;
        rr = rq;
        rn += rq * rq;
        rz_new += rq * rq / Aq;
      }
      rn = block_sum<TB>(rn, red);
      rz_new = block_sum<TB>(rz_new, red);
      if (rn <= a.tol2 * bb) break;
      const double beta = rz_new / rz;
      rz = rz_new;
      if (on) sP[node] = rr / Aq + beta * sP[node];
      __syncthreads();
    }
  }
  if (t == 0 && bb > 0.0 && !(rn <= a.accept2 * bb)) atomicOr(a.err, kErrSolve);
  if (on) sst[node] = kCoreB;
  __syncthreads();
  return true;
}

// ---- the same solve with the system held in LDS.  A system whose cycle
// core fits the one-wave CG is loaded once (node data, and each entry's other
// end as an index into the system's list), peeled, solved and
// back-substituted, and only z at the system's entries is written back (from
// y and the entry records); any other system is flagged in spill and left to
// k_tree_solve.  The arithmetic is that of k_tree_solve: the same
// elimination rule (ties broken by CSR position), sums in entry order, the
// same back substitution and core CG, so either kernel gives the same y.
// Three layouts, one launch each: up to kLdsNodes nodes and kLdsEntries
// entries with everything in LDS (38 bytes per node); up to kLdsNodesLarge
// nodes with each node's first position read from its record instead (34
// bytes per node); and up to kHybNodes nodes and kHybEntries entries with A,
// b and the parent weight in global memory too (10 bytes of LDS per node:
// the graph, the states and the lists), which also runs the block CG for a
// core of up to TB nodes.  The later launches take only the systems an
// earlier one flagged for them (spill code 1: too large, or a core above
// kWaveCore nodes; code 2 is a core no LDS layout takes, or an entry outside
// the system, for k_tree_solve).
constexpr int kLdsNodes = 3840;
constexpr int kLdsNodesLarge = 4288;
constexpr int kLdsEntries = 8192;
constexpr int kHybNodes = 10240;
constexpr int kHybEntries = 20480;
constexpr uint8_t kLActive = 255, kLCore = 254;
constexpr uint16_t kLNoPar = 0xFFFF;

template <int TB, int NODES, int ENTRIES, bool POS_LDS, bool VAL_LDS>
__global__ __launch_bounds__(TB) void k_tree_lds(SolveArgs a, int32_t min_nodes) {
  static_assert(ENTRIES % TB == 0 && kMaxRounds < kLCore && NODES < kLNoPar &&
                    ENTRIES < 0xFFFF && (VAL_LDS || !POS_LDS),
                "LDS solver shape");
  __shared__ double sA_sh[VAL_LDS ? NODES : 1], sB_sh[VAL_LDS ? NODES : 1],
      sW_sh[VAL_LDS ? NODES : 1];
  __shared__ int32_t gpos_sh[POS_LDS ? NODES : 1];
  __shared__ uint16_t eoff[NODES + 2];
  __shared__ uint16_t snb[ENTRIES];
  __shared__ uint16_t spar[NODES];
  __shared__ uint8_t sst[NODES], snst[NODES];
  __shared__ __attribute__((aligned(16))) uint16_t lst[2][NODES];
  __shared__ int32_t scan[TB / 64];
  __shared__ double red[VAL_LDS ? 1 : TB / 64];
  __shared__ int32_t cpos[VAL_LDS ? 1 : TB];
  __shared__ int flag;
  const int t = threadIdx.x;
  const int64_t sys_id = blockIdx.x;
  const int32_t off = a.sys[sys_id * a.nb];
  const int32_t N = a.sys[(sys_id + 1) * a.nb] - off;
  if (min_nodes > 0) {
    // a retry of the systems flagged for their size only
    if (a.lds_off || a.spill[sys_id] != 1 || N < min_nodes || N > NODES) return;
  } else if (N <= 0 || N > NODES || a.lds_off) {
    if (t == 0) a.spill[sys_id] = N > 0 ? 1 : 0;
    return;
  }
  // A, b (then y) and the weight to the parent of node i: LDS, or global
  // memory at the system's list offsets
  double* sA;
  double* sB;
  double* sW;
  if constexpr (VAL_LDS) {
    sA = sA_sh;
    sB = sB_sh;
    sW = sW_sh;
  } else {
    sA = a.A + off;
    sB = a.b + off;
    sW = a.Wp + off;
  }
  // first CSR position of node i
  auto gpos = [&](int32_t i) -> int32_t {
    if constexpr (POS_LDS) return gpos_sh[i];
    else return a.nrec[off + i].q;
  };

  // ---- 1. nodes (first position, entry count clamped above kLdsEntries, A,
  // b) from the list-ordered records, one coalesced stream per system, then
  // the entry offsets by an exclusive scan over contiguous chunks
  if constexpr (VAL_LDS) {
    constexpr int KN = (NODES + TB - 1) / TB;
    NodeRec nr[KN];
#pragma unroll
    for (int u = 0; u < KN; ++u) {
      const int32_t i = t + u * TB;
      if (i < N) nr[u] = a.nrec[off + i];
    }
#pragma unroll
    for (int u = 0; u < KN; ++u) {
      const int32_t i = t + u * TB;
      if (i >= N) continue;
      if constexpr (POS_LDS) gpos_sh[i] = nr[u].q;
      eoff[i] = (uint16_t)min(nr[u].ne, ENTRIES + 1);
      sA[i] = nr[u].A;
      sB[i] = nr[u].b;
      sst[i] = kLActive;
      snst[i] = kLActive;
    }
  } else {
    for (int32_t i = t; i < N; i += TB) {
      const NodeRec nr = a.nrec[off + i];
      eoff[i] = (uint16_t)min(nr.ne, ENTRIES + 1);
      sA[i] = nr.A;
      sB[i] = nr.b;
      sst[i] = kLActive;
      snst[i] = kLActive;
    }
  }
  __syncthreads();
  int32_t total;
  {
    const int lane = t & 63, w = t >> 6;
    const int32_t per = (N + TB - 1) / TB;
    const int32_t k0 = t * per, k1 = min(N, k0 + per);
    int32_t cnt = 0;
    for (int32_t k = k0; k < k1; ++k) cnt += eoff[k];
    int32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    if (lane == 63) scan[w] = incl;
    __syncthreads();
    int32_t before = 0;
    total = 0;
#pragma unroll
    for (int v = 0; v < TB / 64; ++v) {
      const int32_t x = scan[v];
      if (v < w) before += x;
      total += x;
    }
    if (total <= ENTRIES) {
      int32_t o = before + incl - cnt;
      for (int32_t k = k0; k < k1; ++k) {
        const int32_t x = eoff[k];
        eoff[k] = (uint16_t)o;
        o += x;
      }
      if (t == 0) eoff[N] = (uint16_t)total;
    }
  }
  if (total > ENTRIES) {
    if (t == 0) a.spill[sys_id] = 1;
    return;
  }
  __syncthreads();

  // ---- 2. each entry's other end as an index into the list: the loads of
  // a thread's (at most kLdsEntries / TB) entries are all issued before the
  // first is used.  The thread keeps its entries' weights and signed
  // residuals in registers until it writes their z.
  constexpr int KE = VAL_LDS ? ENTRIES / TB : 1;
  double ew[KE], ers[KE];
  int32_t enode[KE];  // the node of each of the thread's entries
  auto node_of = [&](int32_t x) {  // the node of entry x: last i with eoff[i] <= x
    int32_t lo = 0, hi = N - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (eoff[mid] <= x) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  if constexpr (!VAL_LDS) {
    // one entry per thread at a time; the epilogue reads the records again
    int bad = 0;
    for (int32_t x = t; x < total; x += TB) {
      const int32_t lo = node_of(x);
      const int32_t other = a.lidx[a.ent[gpos(lo) + (x - eoff[lo])].nbr];
      if ((uint32_t)other >= (uint32_t)N) bad = 1;
      else snb[x] = (uint16_t)other;
    }
    if (__syncthreads_or(bad)) {
      if (t == 0) a.spill[sys_id] = 2;
      return;
    }
  } else {
    int32_t other[KE];
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      const int32_t x = t + u * TB;
      other[u] = 0;
      ew[u] = ers[u] = 0.0;
      enode[u] = 0;
      if (x < total) {
        const int32_t lo = node_of(x);
        enode[u] = lo;
        const ERec en = a.ent[gpos(lo) + (x - eoff[lo])];
        other[u] = en.nbr;
        ew[u] = en.w;
        ers[u] = en.rs;
      }
    }
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      const int32_t x = t + u * TB;
      if (x < total) other[u] = a.lidx[other[u]];
    }
    // every entry of a listed node ends at a listed node of the same system;
    // anything else leaves the system to k_tree_solve
    int bad = 0;
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      const int32_t x = t + u * TB;
      if (x >= total) continue;
      if ((uint32_t)other[u] >= (uint32_t)N) bad = 1;
      else snb[x] = (uint16_t)other[u];
    }
    if (__syncthreads_or(bad)) {
      if (t == 0) a.spill[sys_id] = 2;
      return;
    }
  }
  uint16_t* act = lst[0];
  uint16_t* nxt = lst[1];
  for (int32_t i = t; i < N; i += TB) act[i] = (uint16_t)i;
  __syncthreads();

  // ---- 3. peeling rounds (a node eliminated in round r keeps state r)
  int32_t nl = N;
  int rounds = 0;
  for (; rounds < a.max_rounds && nl > 0; ++rounds) {
    int changed = 0;
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t i = act[k];
      const int32_t e0 = eoff[i], e1 = eoff[i + 1];
      int32_t p0 = -1;
      bool multi = false;
      for (int32_t x = e0; x < e1; ++x) {
        const int32_t pn = snb[x];
        if (sst[pn] != kLActive) continue;
        if (p0 < 0) {
          p0 = pn;
        } else if (pn != p0) {
          multi = true;
          break;
        }
      }
      uint8_t ns = kLActive;
      if (p0 < 0) {
        ns = (uint8_t)rounds;  // isolated: solved directly
        spar[i] = kLNoPar;
      } else if (!multi) {
        bool p0_other = false;
        for (int32_t x = eoff[p0]; x < eoff[p0 + 1]; ++x) {
          const int32_t pn = snb[x];
          if (pn != i && sst[pn] == kLActive) {
            p0_other = true;
            break;
          }
        }
        const int32_t qi = gpos(i);
        if (p0_other || qi > gpos(p0)) {
          ns = (uint8_t)rounds;
          spar[i] = (uint16_t)p0;
          // weight to the parent: its entries' weights in entry order
          double W = 0.0;
          bool first = true;
          for (int32_t x = e0; x < e1; ++x) {
            if (snb[x] != p0) continue;
            const double wv = a.ent[qi + (x - e0)].w;
            W = first ? wv : W + wv;
            first = false;
          }
          sW[i] = W;
        }
      }
      snst[i] = ns;
      changed |= (ns != kLActive);
    }
    changed = __syncthreads_or(changed);
    if (!changed) break;
    // parents gather the Schur updates of this round's leaves
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t i = act[k];
      if (snst[i] != kLActive) continue;
      const int32_t e0 = eoff[i], e1 = eoff[i + 1];
      double dA = 0.0, db = 0.0;
      for (int32_t x = e0; x < e1; ++x) {
        const int32_t pn = snb[x];
        if (snst[pn] != rounds || spar[pn] != i) continue;
        bool first = true;
        for (int32_t f = e0; f < x; ++f)
          if (snb[f] == pn) {
            first = false;
            break;
          }
        if (!first) continue;
        const double Ap = sA[pn], Wn = sW[pn];
        dA += Wn * Wn / Ap;
        db += Wn * sB[pn] / Ap;
      }
      sA[i] -= dA;
      sB[i] += db;
    }
    __syncthreads();
    for (int32_t k = t; k < nl; k += TB) sst[act[k]] = snst[act[k]];
    __syncthreads();
    nl = block_compact<TB>(
        nl, [&](int32_t k) { return sst[act[k]] == kLActive; }, [&](int32_t k) { return act[k]; },
        nxt, scan);
    uint16_t* tmp = act;
    act = nxt;
    nxt = tmp;
  }
  __syncthreads();

  // ---- 4. the cycle core: one-wave CG up to kWaveCore nodes; a larger core
  // of up to TB nodes gets the block CG in the third layout (the first two
  // flag it for that one, which keeps their registers free); anything else
  // goes to k_tree_solve
  if (nl > 0) {
    if (t == 0) flag = 0;
    __syncthreads();
    if (nl <= kWaveCore) {
      if (t < 64) {
        const bool ok = wave_core_cg_lds(a, act, nl, gpos, eoff, snb, sst, sA, sB,
                                         (double (*)[kWaveNb])nxt,
                                         (int32_t (*)[kWaveNb])(nxt + 4 * kWaveCore * kWaveNb));
        if (t == 0) flag = ok ? 1 : 0;
      }
    } else if (nl <= TB) {
      if constexpr (!VAL_LDS) {
        // p in sW: a core node has no parent weight
        const bool ok = block_core_cg_lds<TB>(a, act, nl, gpos, eoff, snb, sst, sA, sB, sW,
                                              nxt, cpos, red);
        if (t == 0) flag = ok ? 1 : 0;
      }
    }
    __syncthreads();
    if (!flag) {
      if (t == 0) a.spill[sys_id] = (VAL_LDS && nl > kWaveCore && nl <= TB) ? 1 : 2;
      return;
    }
  }

  // ---- 5. back substitution in reverse round order (y replaces b): the
  // nodes of a round, found by their state, are independent of each other
  for (int rnd = rounds - 1; rnd >= 0; --rnd) {
    for (int32_t i = t; i < N; i += TB) {
      if (sst[i] != rnd) continue;
      const int32_t pn = spar[i];
      sB[i] = pn == kLNoPar ? sB[i] / sA[i] : (sB[i] + sW[i] * sB[pn]) / sA[i];
    }
    __syncthreads();
  }
  // z at every entry of the system, one entry per thread as in step 2, both
  // ends' y from the solved b
  const int g = (int)(sys_id % a.L);
  const double zs = g >= a.L_p ? a.zscale_s : 1.0;
  if constexpr (VAL_LDS) {
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      const int32_t x = t + u * TB;
      if (x >= total) continue;
      const int32_t i = enode[u];
      a.zp[gpos(i) + (x - eoff[i])] = signed_z(ers[u], ew[u], sB[i], sB[snb[x]], a.sigma, zs);
    }
  } else {
    for (int32_t x = t; x < total; x += TB) {
      const int32_t i = node_of(x);
      const int32_t f = gpos(i) + (x - eoff[i]);
      const ERec en = a.ent[f];
      a.zp[f] = signed_z(en.rs, en.w, sB[i], sB[snb[x]], a.sigma, zs);
    }
  }
  if (t == 0) a.spill[sys_id] = 0;
}

}  // namespace

// ------------------------------------------------------------------ launchers

int64_t scan_part_size(int64_t len) { return ceil_div(len, kScanChunk) + 1; }

void launch_scan(int32_t* a, int64_t len, int32_t* part, hipStream_t s) {
  if (len <= 0) return;
  const int64_t nb = ceil_div(len, kScanChunk);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanTB), 0, s, a, len, part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTB), 0, s, part, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanTB), 0, s, a, len, part);
}

void launch_select(const CatView& cat, int C, int64_t n, const int64_t* idx, uint64_t seed,
                   const int64_t* steps, int64_t step_scalar, int chain0, BatchBufs b,
                   int* err_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(grid_for((int64_t)C * n)), dim3(kBlock), 0, s, cat, C, n, idx,
                     (uint32_t)seed, (uint32_t)(seed >> 32), steps, step_scalar, chain0, b,
                     err_flag);
}

BucketShape bucket_shape(int64_t C, int64_t n, int64_t M) {
  BucketShape bs;
  // about kBucketTarget / 2 .. kBucketTarget entries per bucket on average
  // (2 n 2^sb / M per chain): few enough buckets that the scatter writes runs
  // of records, one workgroup of kSortTB threads per bucket
  int sb = 0;
  while (sb < kBucketMaxSB && (2 * n << (sb + 1)) / std::max<int64_t>(M, 1) <= kBucketTarget) ++sb;
  while (sb < kBucketMaxSB && ceil_div(M, (int64_t)1 << sb) > kBucketMax) ++sb;
  bs.sb = sb;
  bs.nbk = ceil_div(M, (int64_t)1 << sb);
  bs.nb = C * bs.nbk;
  bs.hb = std::max<int64_t>(ceil_div(2 * n, kBucketHB), 1);  // counting blocks per chain
  bs.words = C * bs.hb * bs.nbk + bs.nb + 1;
  bs.ok = bs.nbk <= kBucketMax;
  return bs;
}

template <int RPT>
void launch_bucket_sort(const BucketShape& bs, int M, const int32_t* base, const BatchBufs& b,
                        hipStream_t s) {
  const size_t lds = (size_t)RPT * kSortTB * 8 + (size_t)2 * (((size_t)1 << bs.sb) + 1) * 4;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_bucket_sort<RPT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_bucket_sort<RPT>, dim3((unsigned)bs.nb), dim3(kSortTB), lds, s, bs.nbk, bs.sb,
                     M, base, b);
}

void launch_build_csr(const CatView& cat, int C, int64_t n, BatchBufs b, int32_t* bucket_buf,
                      int32_t* scan_part, hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  const BucketShape bs = bucket_shape(C, n, cat.M);
  int32_t* counts = bucket_buf;                         // [C][hb][nbk]
  int32_t* tot = bucket_buf + (int64_t)C * bs.hb * bs.nbk;  // [nb + 1] totals, then bases
  const size_t lds_count = (size_t)bs.nbk * 4;
  const dim3 grid((unsigned)bs.hb, (unsigned)C);
  hipLaunchKernelGGL(k_bucket_count, grid, dim3(kBucketTB), lds_count, s, n, bs.sb, bs.nbk,
                     (const int32_t*)b.ev, counts);
  hipLaunchKernelGGL(k_bucket_prefix, dim3(grid_for(bs.nb)), dim3(kBlock), 0, s, bs.nbk, bs.nb,
                     bs.hb, counts, tot, b.start, (int64_t)C * cat.M, E);
  launch_scan(tot, bs.nb + 1, scan_part, s);
  hipLaunchKernelGGL(k_bucket_scatter, grid, dim3(kBucketTB), lds_count, s, n, bs.sb, bs.nbk,
                     (const int32_t*)counts, (const int32_t*)tot, b);
  // records held per thread: room for three times the average bucket, 2,048
  // to 16,384 (a larger bucket is sorted in global memory)
  const int64_t need = 3 * ceil_div(E, bs.nb);
  if (need <= 4 * kSortTB) launch_bucket_sort<4>(bs, cat.M, tot, b, s);
  else if (need <= 8 * kSortTB) launch_bucket_sort<8>(bs, cat.M, tot, b, s);
  else if (need <= 16 * kSortTB) launch_bucket_sort<16>(bs, cat.M, tot, b, s);
  else launch_bucket_sort<32>(bs, cat.M, tot, b, s);
}

void launch_phase_rows(const CatView& cat, int64_t E, BatchBufs b, int32_t* flags,
                       int32_t* scan_part, int64_t* n_p, hipStream_t s) {
  hipLaunchKernelGGL(k_phase_flags, dim3(grid_for(E + 1)), dim3(kBlock), 0, s, E, b, cat.L_p,
                     flags);
  launch_scan(flags, E + 1, scan_part, s);
  hipLaunchKernelGGL(k_phase_rows, dim3(grid_for(E)), dim3(kBlock), 0, s, E, b, cat.L_p, flags,
                     n_p);
}

void launch_assemble(const CatView& cat, const NetView& net, const NetView& net_s, int C, int64_t n,
                     const double* theta, int64_t theta_stride, const int32_t* rows, BatchBufs b,
                     bool grad64, int32_t* act_clear, hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(E)), dim3(kBlock), 0, s, cat, net, net_s, n, theta,
                     theta_stride, rows, E, b, grad64, act_clear);
}

void launch_residual(const CatView& cat, int C, int64_t n, const double* theta,
                     int64_t theta_stride, int whiten, BatchBufs b, SolveBufs sv, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for((int64_t)C * n)), dim3(kBlock), 0, s, cat, C, n,
                     theta, theta_stride, whiten, b, sv.act);
}

int64_t list_blocks(int64_t C, int64_t n, int64_t L) {
  int64_t nb = ceil_div(2 * n, 4096);
  const int64_t cap = ((int64_t)1 << 22) / (C * L);
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : nb;
}

int64_t list_block_span(int64_t n, int64_t nb) { return ceil_div(2 * n, nb); }

hipError_t exact_whiten(const CatView& cat, int C, int64_t n, BatchBufs b, SolveBufs sv, int* err,
                        hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  const int64_t S = (int64_t)C * cat.L;
  const int64_t nb = list_blocks(C, n, cat.L), span = list_block_span(n, nb);
  const double lambda = (cat.sigma * cat.sigma) / (cat.kappa * cat.kappa);
  const size_t lds = (size_t)cat.L * 4;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_list_count,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_list_fill, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_list_count, dim3((unsigned)nb, (unsigned)C), dim3(kListTB), lds, s, n,
                     cat.L, nb, span, b, sv);
  launch_scan(sv.sys, S * nb + 1, sv.scan_part, s);
  hipLaunchKernelGGL(k_list_fill, dim3((unsigned)nb, (unsigned)C), dim3(kListTB), lds, s, n, cat.L,
                     nb, span, lambda, E, b, sv);
  SolveArgs a;
  a.nend = b.nend;
  a.ent = sv.ent;
  a.sys = sv.sys;
  a.nb = nb;
  a.list = sv.list;
  a.A = sv.vec;
  a.b = sv.vec + E;
  a.y = sv.vec + 2 * E;
  a.Wp = sv.vec + 3 * E;
  a.rr = sv.vec + 4 * E;
  a.p = sv.vec + 5 * E;
  a.ap = sv.vec + 6 * E;
  a.state = sv.ivec;
  a.nstate = sv.ivec + E;
  a.par = sv.ivec + 2 * E;
  a.next = sv.ivec + 3 * E;
  a.elim = sv.ivec + 4 * E;
  a.lambda = lambda;
  a.max_rounds = kMaxRounds;
  // CG to a relative residual of 1e-16 (z = (r - U y)/sigma^2 scales y
  // errors by 1/sigma^2, so y is solved to FP64 rounding), at most 1,000
  // iterations per pass and three passes; a core still above 1e-8 after them
  // is an error
  a.max_iter = 1000;
  a.tol2 = 1e-32;
  a.accept2 = 1e-16;
  a.err = err;
  a.lidx = sv.lidx;
  a.nrec = sv.nrec;
  a.spill = sv.spill;
  a.zp = b.zp;
  a.sigma = cat.sigma;
  a.zscale_s = cat.zscale_s;
  a.L = cat.L;
  a.L_p = cat.L_p;
  const char* tg = std::getenv("SPIDER_TREE_GLOBAL");
  a.lds_off = (tg && tg[0] == '1') ? 1 : 0;
  hipLaunchKernelGGL((k_tree_lds<kTreeBlock, kLdsNodes, kLdsEntries, true, true>),
                     dim3((unsigned)S), dim3(kTreeBlock), 0, s, a, 0);
  hipLaunchKernelGGL((k_tree_lds<kTreeBlock, kLdsNodesLarge, kLdsEntries, false, true>),
                     dim3((unsigned)S), dim3(kTreeBlock), 0, s, a, kLdsNodes + 1);
  hipLaunchKernelGGL((k_tree_lds<kTreeBlock, kHybNodes, kHybEntries, false, false>),
                     dim3((unsigned)S), dim3(kTreeBlock), 0, s, a, 1);
  hipLaunchKernelGGL(k_tree_solve<kTreeBlock>, dim3((unsigned)S), dim3(kTreeBlock), 0, s, a);
  return hipGetLastError();
}

int64_t reduce_part_bytes(int64_t E) { return (ceil_div(E, 64) + 1) * 2 * (int64_t)sizeof(double4); }

void launch_reduce(const CatView& cat, int C, int64_t n, double scale, BatchBufs b, double* G,
                   void* part, hipStream_t s) {
  const int64_t K = (int64_t)C * cat.M, E = 2 * (int64_t)C * n;
  hipLaunchKernelGGL(k_reduce_waves, dim3((unsigned)ceil_div(E, kReduceTB)), dim3(kReduceTB), 0, s,
                     E, n, cat.M, scale, b, G, (double4*)part);
  hipLaunchKernelGGL(k_reduce_keys, dim3(grid_for(K)), dim3(kBlock), 0, s, K, b, G,
                     (const double4*)part);
}

void launch_obs_z(int64_t Q, const BatchBufs& b, hipStream_t s) {
  if (Q <= 0) return;
  hipLaunchKernelGGL(k_obs_z, dim3(grid_for(Q)), dim3(kBlock), 0, s, Q, b);
}

void launch_batch_terms_out(int64_t n, const BatchBufs& b, const double* theta, double* T_i,
                            double* T_j, double* gT_i, double* gT_j, double* r, double* z,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_batch_terms_out, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b, theta, T_i,
                     T_j, gT_i, gT_j, r, z);
}

void launch_linear_keep(const BatchBufs& b, const double* theta, int64_t n, double e_max,
                        uint8_t* keep, unsigned long long* count, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_linear_keep, dim3(grid_for(n)), dim3(kBlock), 0, s, b, theta, n, e_max,
                     keep, count);
}

}  // namespace spider
