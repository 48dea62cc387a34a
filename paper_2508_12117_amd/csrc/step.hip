// Per-step kernels of the hot path other than the travel-time network, and
// the catalog preparation done once at load.
//
//   select    minibatch without replacement (Sec. 3.2) and its gathers
//   residual  T = |x - s|/v0 softplus(o)/ln2 and dT/dx in FP64 from the
//             network outputs; r = tau - [T_i - T_j + t_i - t_j] (Eq. 1)
//   whitening z = Sigma_B^{-1} r (Sec. 3.1, eq:marginal_sigma): diagonal, or
//             exact by Woodbury + preconditioned CG per (chain, group)
//   reduce    per-event gradient sum over a sorted (chain, event) list:
//             every event's terms are contiguous, summed in a fixed order by
//             one thread, no floating-point atomics (deterministic)
//   centroid  per-chain mean of theta (fixed-order two-level reduction)
//   update    priors + SGLD / pSGLD (eq:pSGLD) + Philox noise + Welford
#include <climits>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "device_rng.h"
#include "internal.h"

namespace spider {

namespace {

constexpr int kBlock = 256;
constexpr double kLn2 = 0.69314718055994530941723212145818;

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
    const int64_t t = steps ? steps[c] : step_scalar;
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
  b.obs[q] = o;
  b.ev[2 * q] = rc.i;
  b.ev[2 * q + 1] = rc.j;
  b.sta[2 * q] = rc.g;
  b.sta[2 * q + 1] = rc.g;
  b.tau[q] = (double)rc.dt;
  b.w[q] = rc.w;
}

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

// Travel time and source gradient of one row from the network output.
__device__ inline void assemble_tt(const NetView& net, const double x[3], const double s[3],
                                   const RowOut& no, double& T, double g[3]) {
  const double d0 = x[0] - s[0], d1 = x[1] - s[1], d2 = x[2] - s[2];
  const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double T0 = dist / net.v0;
  const double o = (double)no.o;
  const double sp = fmax(o, 0.0) + log1p(exp(-fabs(o)));      // softplus
  const double sg = o >= 0.0 ? 1.0 / (1.0 + exp(-o)) : exp(o) / (1.0 + exp(o));  // sigmoid
  const double f = sp / kLn2;
  T = T0 * f;
  const double a = f / (net.v0 * dist);
  const double bsc = T0 * sg / kLn2;
  g[0] = a * d0 + bsc * ((double)no.d0 * net.inv_half[0]);
  g[1] = a * d1 + bsc * ((double)no.d1 * net.inv_half[1]);
  g[2] = a * d2 + bsc * ((double)no.d2 * net.inv_half[2]);
}

__global__ void k_residual(CatView cat, NetView net, NetView net_s, int C, int64_t n,
                           const double* theta, int64_t theta_stride, int whiten, BatchBufs b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)C * n) return;
  double T[2], tt[2];
  const bool s_phase = b.sta[2 * q] >= cat.L_p;
  for (int side = 0; side < 2; ++side) {
    const int64_t row = 2 * q + side;
    const double4 xe = b.xt[row];  // the row's event state, as the network read it
    const double* st = cat.stations + (int64_t)b.sta[row] * 3;
    const double x[3] = {xe.x, xe.y, xe.z};
    const double s[3] = {st[0], st[1], st[2]};
    double g[3];
    assemble_tt(s_phase ? net_s : net, x, s, b.net_out[row], T[side], g);
    b.T[row] = T[side];
    b.gT[row * 3 + 0] = g[0];
    b.gT[row * 3 + 1] = g[1];
    b.gT[row * 3 + 2] = g[2];
    tt[side] = xe.w;
  }
  const double r = b.tau[q] - ((T[0] - T[1]) + (tt[0] - tt[1]));
  b.r[q] = r;
  const double s2 = cat.sigma * cat.sigma;
  if (whiten == kWhitenL1) {
    b.z[q] = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);  // d|r|/dr, 0 at 0
  } else if (whiten == 0 || cat.kappa == 0.0) {
    b.z[q] = r / s2 * (s_phase ? cat.zscale_s : 1.0);
  } else if (whiten == 1) {
    b.z[q] = r / (s2 + 2.0 * cat.kappa * cat.kappa * b.w[q]) * (s_phase ? cat.zscale_s : 1.0);
  } else {
    b.wr[q] = make_double2(b.w[q], r);  // exact whitening: the solver's edge gathers
  }
}

// ---- exact whitening: Sigma_B = s2 I + k2 U U^T, U = W^{1/2} A_B.
// z = (r - U y)/s2 with (lambda I + U^T U) y = U^T r, lambda = s2/k2.  U^T U
// is the w-weighted Laplacian of the batch's event graph in each group, so
// the system is block diagonal over (chain, group); each block is solved by
// Jacobi-preconditioned CG in FP64 by one workgroup.

// Sort keys are 32-bit whenever the key range fits (half the sort traffic),
// else 64-bit.
template <class K>
__global__ void k_group_keys(int C, int64_t n, int M, int L, const BatchBufs b, K* keys,
                             uint32_t* vals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * (int64_t)C * n) return;
  const int64_t c = (e >> 1) / n;
  keys[e] = (K)(((uint64_t)(c * L + b.sta[e]) * (uint64_t)M) + (uint64_t)b.ev[e]);
  vals[e] = (uint32_t)e;
}

template <class K>
__global__ void k_heads(const K* keys, int64_t E, int32_t* flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= E) return;
  flags[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

// After an inclusive scan of the head flags (flags -> node number + 1).
template <class K>
__global__ void k_nodes(const K* keys, const uint32_t* vals, const int32_t* scan, int64_t E,
                        int M, int32_t* node_of, int32_t* node_start, int32_t* seg_begin,
                        int32_t* seg_end, int32_t* count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= E) return;
  const int32_t node = scan[p] - 1;
  node_of[vals[p]] = node;
  const bool head = p == 0 || keys[p] != keys[p - 1];
  if (head) {
    node_start[node] = (int32_t)p;
    const K seg = keys[p] / (K)M;
    if (p == 0 || keys[p - 1] / (K)M != seg) seg_begin[seg] = node;
  }
  const bool tail = p == E - 1 || keys[p + 1] != keys[p];
  if (tail) {
    const K seg = keys[p] / (K)M;
    if (p == E - 1 || keys[p + 1] / (K)M != seg) seg_end[seg] = node + 1;
  }
  if (p == E - 1) {
    node_start[node + 1] = (int32_t)E;
    *count = node + 1;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

struct SolveArgs {
  const uint32_t* vals;       // entries sorted by (chain, group, event)
  const int32_t* node_of;     // node of each entry
  const int32_t* nbr;         // per sorted entry: the node at the other end of its edge
  const double* wgt;          // per sorted entry: the edge weight w
  const int32_t* node_start;  // entries of node q: [node_start[q], node_start[q + 1])
  const int32_t* seg_begin;
  const int32_t* seg_end;
  const double* w;
  const double* r;
  double* A;        // diagonal, Schur-updated as leaves are eliminated
  double* b;        // right-hand side, Schur-updated
  double* y;        // solution
  double* Wp;       // weight to the parent at elimination
  double* rr;       // CG vectors for the nodes left on cycles
  double* p;
  double* ap;
  int32_t* state;   // kActive, or the round in which the node was removed
  int32_t* nstate;
  int32_t* par;     // parent of an eliminated node (-1: solved on its own)
  int32_t* core;    // scratch: active-node list (room for one entry per node)
  int32_t* core2;   // scratch: second active-node list, then the elimination order
                    // (room for 2 n_entries)
  int32_t n_entries;
  double lambda;
  int max_rounds;
  int max_iter;
  double tol2;     // CG stops once |res|^2 <= tol2 |rhs|^2
  double accept2;  // after max_iter, |res|^2 > accept2 |rhs|^2 raises kErrSolve
  int* err;        // error bits of the step
};

constexpr int32_t kActive = -1;
constexpr int kMaxRounds = 64;
constexpr int kTreeBlock = 1024;  // threads per (chain, group) system

// Neighbour node, weight and right-hand-side term (+-sqrt(w) r, the entry's
// row of U^T r) of every sorted entry, so that the node kernels and the
// elimination rounds read them contiguously instead of through a chain of
// lookups.
__global__ void k_edges(int64_t E, const uint32_t* vals, const int32_t* node_of, const double2* wr,
                        int32_t* nbr, double* wgt, double* rv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const uint32_t en = vals[e];
  const double2 x = wr[en >> 1];  // (w, r) of the entry's observation
  nbr[e] = node_of[en ^ 1u];
  wgt[e] = x.x;
  rv[e] = ((en & 1u) ? -1.0 : 1.0) * sqrt(x.x) * x.y;
}
constexpr int32_t kCore = 1 << 30;  // solved by CG after the peeling rounds
constexpr int32_t kPair = -2;       // solved directly: an isolated single edge


// Appends, in order, the n items item(k) that satisfy keep(k) to out (fixed
// order: per-wave ballot, then a block-wide prefix over the waves); returns
// the number appended.  All threads of the block call it.
template <int TB, class Keep, class Item>
__device__ int32_t block_compact(int32_t n, Keep&& keep, Item&& item, int32_t* out,
                                 int32_t* warp_base, int32_t* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) *total = 0;
  __syncthreads();
  for (int32_t k0 = 0; k0 < n; k0 += TB) {
    const int32_t k = k0 + t;
    const bool on = k < n && keep(k);
    const uint64_t mask = __ballot(on);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) warp_base[w] = __popcll(mask);
    __syncthreads();
    if (t == 0) {
      int32_t run = *total;
      for (int v = 0; v < TB / 64; ++v) {
        const int32_t cnt = warp_base[v];
        warp_base[v] = run;
        run += cnt;
      }
      *total = run;
    }
    __syncthreads();
    if (on) out[warp_base[w] + before] = item(k);
    __syncthreads();
  }
  // every thread reads the count before any thread can start another call
  // (which resets it)
  const int32_t count = *total;
  __syncthreads();
  return count;
}

// Diagonal lambda + sum w and right-hand side (U^T r)_q of every node, one
// thread per node over all (chain, group) blocks.
__global__ void k_node_init(const int32_t* count, const int32_t* node_start, const double* wgt,
                            const double* rv, double lambda, double* A, double* b, int32_t* state,
                            int32_t* par) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *count) return;
  double rhs = 0.0, dg = lambda;
  for (int32_t e = node_start[q]; e < node_start[q + 1]; ++e) {
    rhs += rv[e];
    dg += wgt[e];
  }
  A[q] = dg;
  b[q] = rhs;
  state[q] = kActive;
  par[q] = -1;
}

// Isolated single edges (both ends have one entry: at minibatch density
// nearly every component) solved directly as 2x2 systems by their smaller
// end, one thread per node.
__global__ void k_pairs(const int32_t* count, const int32_t* node_start, const int32_t* nbr,
                        const double* wgt, const double* A, const double* b, double* y,
                        int32_t* state) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *count) return;
  const int32_t e = node_start[q];
  if (node_start[q + 1] - e != 1) return;
  const int32_t p = nbr[e];
  if (p <= q || node_start[p + 1] - node_start[p] != 1) return;
  const double w = wgt[e], Aq = A[q], Ap = A[p], bq = b[q], bp = b[p];
  const double det = Aq * Ap - w * w;
  y[q] = (Ap * bq + w * bp) / det;
  y[p] = (Aq * bp + w * bq) / det;
  state[q] = kPair;
  state[p] = kPair;
}

// One workgroup per (chain, group) block of (lambda I + L) y = U^T r, after
// k_node_init and k_pairs.
//  0. Isolated single edges are already solved (k_pairs); the other nodes
//     are listed in node order and only they take part in 1-3.
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
template <int TB>
__global__ __launch_bounds__(TB) void k_tree_solve(SolveArgs a) {
  __shared__ double sh[TB];
  __shared__ int32_t warp_base[TB / 64];
  __shared__ int32_t total_sh;
  __shared__ int32_t elim_start[kMaxRounds + 2];  // elimination order: round r's nodes
  const int32_t nb = a.seg_begin[blockIdx.x];
  const int32_t ne = a.seg_end[blockIdx.x];
  if (ne <= nb) return;
  const int t = threadIdx.x;
  // the nodes still active at the start of each round (two buffers in turn),
  // and every eliminated node in round order; all lists keep node order
  int32_t* act = a.core + nb;
  int32_t* act_next = a.core2 + nb;
  int32_t* elim = a.core2 + a.n_entries + nb;
  int32_t nl = block_compact<TB>(
      ne - nb, [&](int32_t k) { return a.state[nb + k] != kPair; }, [&](int32_t k) { return nb + k; },
      act, warp_base, &total_sh);
  int32_t n_elim = 0;

  // ---- 1. peeling rounds over the active nodes
  int rounds = 0;
  for (; rounds < a.max_rounds && nl > 0; ++rounds) {
    if (t == 0) elim_start[rounds] = n_elim;
    // phase 1: classify active nodes
    int changed = 0;
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t q = act[k];
      int32_t p0 = -1;
      double W = 0.0;
      bool multi = false;
      for (int32_t e = a.node_start[q]; e < a.node_start[q + 1]; ++e) {
        const int32_t pn = a.nbr[e];
        if (a.state[pn] != kActive) continue;
        if (p0 < 0) {
          p0 = pn;
          W = a.wgt[e];
        } else if (pn == p0) {
          W += a.wgt[e];
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
        for (int32_t e = a.node_start[p0]; e < a.node_start[p0 + 1]; ++e) {
          const int32_t pn = a.nbr[e];
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
    // phase 2: parents gather the Schur updates of this round's leaves
    for (int32_t k = t; k < nl; k += TB) {
      const int32_t q = act[k];
      if (a.nstate[q] == kActive) {
        const int32_t e0 = a.node_start[q], e1 = a.node_start[q + 1];
        double dA = 0.0, db = 0.0;
        for (int32_t e = e0; e < e1; ++e) {
          const int32_t pn = a.nbr[e];
          if (a.nstate[pn] != rounds || a.par[pn] != q) continue;
          bool first = true;
          for (int32_t f = e0; f < e; ++f)
            if (a.nbr[f] == pn) {
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
    // this round's eliminated nodes join the elimination order; the rest
    // form the next round's active list
    n_elim += block_compact<TB>(
        nl, [&](int32_t k) { return a.state[act[k]] != kActive; }, [&](int32_t k) { return act[k]; },
        elim + n_elim, warp_base, &total_sh);
    nl = block_compact<TB>(
        nl, [&](int32_t k) { return a.state[act[k]] == kActive; }, [&](int32_t k) { return act[k]; },
        act_next, warp_base, &total_sh);
    int32_t* tmp = act;
    act = act_next;
    act_next = tmp;
  }
  if (t == 0) elim_start[rounds] = n_elim;
  __syncthreads();

  // ---- 2. nodes still active sit on cycles (or on paths longer than the
  // round cap): Jacobi-preconditioned CG on them only.  Each pass starts from
  // the true residual b - A y of the current y (the first from y = 0), so
  // later passes correct the drift of CG's recursively updated residual.
  const int32_t* core = act;
  const int32_t ncore = nl;
  if (ncore > 0) {
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
        for (int32_t e = a.node_start[q]; e < a.node_start[q + 1]; ++e) {
          const int32_t pn = a.nbr[e];
          if (a.state[pn] == kActive) v += a.wgt[e] * a.y[pn];
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
          for (int32_t e = a.node_start[q]; e < a.node_start[q + 1]; ++e) {
            const int32_t pn = a.nbr[e];
            if (a.state[pn] == kActive) v -= a.wgt[e] * a.p[pn];
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
    // not converged to the acceptance level: the step reports an error
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
}

__global__ void k_exact_z(int64_t Q, double s2, const double* w, const double* r,
                          const int32_t* node_of, const double* y, const int32_t* sta,
                          int32_t L_p, double zscale_s, double* z) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const double yi = y[node_of[2 * q]];
  const double yj = y[node_of[2 * q + 1]];
  z[q] = (r[q] - sqrt(w[q]) * (yi - yj)) / s2 * (sta[2 * q] >= L_p ? zscale_s : 1.0);
}

// ---- per-event reduction

template <class K>
__global__ void k_event_keys(int C, int64_t n, int M, const BatchBufs b, K* keys,
                             uint32_t* vals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * (int64_t)C * n) return;
  const int64_t c = (e >> 1) / n;
  keys[e] = (K)((uint64_t)c * (uint64_t)M + (uint64_t)b.ev[e]);
  vals[e] = (uint32_t)e;
}

template <class K>
__global__ void k_reduce_runs(const K* keys, const uint32_t* vals, int64_t E, double scale,
                              const BatchBufs b, double* G) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= E) return;
  const K key = keys[p];
  if (p > 0 && keys[p - 1] == key) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t q = p; q < E && keys[q] == key; ++q) {
    const uint32_t e = vals[q];
    const double cz = ((e & 1u) ? -scale : scale) * b.z[e >> 1];
    s0 += cz * b.gT[e * 3 + 0];
    s1 += cz * b.gT[e * 3 + 1];
    s2 += cz * b.gT[e * 3 + 2];
    s3 += cz;
  }
  double* g = G + (uint64_t)key * 4;
  g[0] = s0;
  g[1] = s1;
  g[2] = s2;
  g[3] = s3;
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
  for (int a = 0; a < 4; ++a) {
    double s = 0.0;
    for (int64_t m = m0 + threadIdx.x; m < m1; m += kBlock) s += th[m * 4 + a];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[((int64_t)c * nchunk + chunk) * 4 + a] = s;
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

__global__ void k_batch_terms_out(int64_t n, BatchBufs b, double* Ti, double* Tj, double* gi,
                                  double* gj, double* r, double* z) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  if (Ti) Ti[q] = b.T[2 * q];
  if (Tj) Tj[q] = b.T[2 * q + 1];
  for (int a = 0; a < 3; ++a) {
    if (gi) gi[q * 3 + a] = b.gT[(2 * q) * 3 + a];
    if (gj) gj[q * 3 + a] = b.gT[(2 * q + 1) * 3 + a];
  }
  if (r) r[q] = b.r[q];
  if (z) z[q] = b.z[q];
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

// Linear-regime test of the n slots of one chain's batch (rows 2q, 2q + 1 =
// events i, j): dT = T_j - T_i, lin = grad T(x_i) . (x_j - x_i), keep[q] =
// |dT - lin| <= e_max |dT|; the kept count is added to *count.
__global__ void k_linear_keep(const BatchBufs b, const double* theta, int64_t n, double e_max,
                              uint8_t* keep, unsigned long long* count) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned int k = 0;
  if (q < n) {
    const double* xi = theta + (int64_t)b.ev[2 * q] * 4;
    const double* xj = theta + (int64_t)b.ev[2 * q + 1] * 4;
    const double* g = b.gT + 6 * q;
    const double dT = b.T[2 * q + 1] - b.T[2 * q];
    const double lin = g[0] * (xj[0] - xi[0]) + g[1] * (xj[1] - xi[1]) + g[2] * (xj[2] - xi[2]);
    k = fabs(dT - lin) <= e_max * fabs(dT) ? 1u : 0u;
    keep[q] = (uint8_t)k;
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

void launch_select(const CatView& cat, int C, int64_t n, const int64_t* idx, uint64_t seed,
                   const int64_t* steps, int64_t step_scalar, int chain0, BatchBufs b,
                   int* err_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(grid_for((int64_t)C * n)), dim3(kBlock), 0, s, cat, C, n, idx,
                     (uint32_t)seed, (uint32_t)(seed >> 32), steps, step_scalar, chain0, b,
                     err_flag);
}

void launch_residual(const CatView& cat, const NetView& net, const NetView& net_s, int C, int64_t n,
                     const double* theta, int64_t theta_stride, int whiten, BatchBufs b,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for((int64_t)C * n)), dim3(kBlock), 0, s, cat, net,
                     net_s, C, n, theta, theta_stride, whiten, b);
}

namespace {
struct PhaseIsP {
  const int32_t* sta;
  int32_t L_p;
  __device__ bool operator()(int32_t row) const { return sta[row] < L_p; }
};

__global__ void k_scatter_rows(const RowOut* compact, const int32_t* list, int64_t E,
                               RowOut* out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < E) out[list[v]] = compact[v];
}
}  // namespace

hipError_t partition_rows_by_phase(const int32_t* sta, int32_t L_p, int64_t E, int32_t* list,
                                   uint64_t* count, void* temp, size_t* temp_bytes,
                                   hipStream_t s) {
  return rocprim::partition(temp, *temp_bytes, rocprim::counting_iterator<int32_t>(0), list,
                            count, (size_t)E, PhaseIsP{sta, L_p}, s);
}

void launch_scatter_rows(const RowOut* compact, const int32_t* list, int64_t E, RowOut* out,
                         hipStream_t s) {
  if (E == 0) return;
  hipLaunchKernelGGL(k_scatter_rows, dim3(grid_for(E)), dim3(kBlock), 0, s, compact, list, E,
                     out);
}

size_t sort_temp_bytes(int64_t entries) {
  size_t bytes = 0, bytes32 = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                            (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)entries, 0, 64,
                            (hipStream_t)0);
  (void)rocprim::radix_sort_pairs(nullptr, bytes32, (uint32_t*)nullptr, (uint32_t*)nullptr,
                            (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)entries, 0, 32,
                            (hipStream_t)0);
  if (bytes32 > bytes) bytes = bytes32;
  size_t scan = 0;
  (void)rocprim::inclusive_scan(nullptr, scan, (int32_t*)nullptr, (int32_t*)nullptr, (size_t)entries,
                          rocprim::plus<int32_t>(), (hipStream_t)0);
  return bytes > scan ? bytes : scan;
}

static int bits_for(uint64_t maxval) {
  int b = 1;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

// Entries sorted by (chain, group, event) with K-bit keys; runs of equal keys
// become the nodes of the (chain, group) systems: node_of per entry,
// node_start, the node range of every (chain, group) and the node count.
template <class K>
hipError_t group_nodes(int C, int64_t n, const CatView& cat, const BatchBufs& b,
                       const SortBufs& sb, int end_bit, hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  K* key_in = (K*)sb.key_in;
  K* key_out = (K*)sb.key_out;
  hipLaunchKernelGGL(k_group_keys<K>, dim3(grid_for(E)), dim3(kBlock), 0, s, C, n, cat.M, cat.L,
                     b, key_in, sb.val_in);
  size_t tb = sb.temp_bytes;
  hipError_t e = rocprim::radix_sort_pairs(sb.temp, tb, key_in, key_out, sb.val_in, sb.val_out,
                                           (size_t)E, 0, end_bit, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_heads<K>, dim3(grid_for(E)), dim3(kBlock), 0, s, key_out, E, sb.flags);
  int32_t* scan = (int32_t*)sb.key_in;  // key_in is free after the sort
  tb = sb.temp_bytes;
  e = rocprim::inclusive_scan(sb.temp, tb, sb.flags, scan, (size_t)E, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)C * cat.L)), dim3(kBlock), 0, s,
                     sb.seg_begin, 0, (int64_t)C * cat.L);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)C * cat.L)), dim3(kBlock), 0, s,
                     sb.seg_end, 0, (int64_t)C * cat.L);
  hipLaunchKernelGGL(k_nodes<K>, dim3(grid_for(E)), dim3(kBlock), 0, s, key_out, sb.val_out, scan,
                     E, cat.M, sb.node_of, sb.node_start, sb.seg_begin, sb.seg_end, sb.count);
  return hipGetLastError();
}

hipError_t exact_whiten(const CatView& cat, int C, int64_t n, BatchBufs b, SortBufs sb, int* err,
                        hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  if (E <= 0) return hipSuccess;  // the node kernels read the node count k_nodes writes
  const int end_bit = bits_for((uint64_t)C * cat.L * (uint64_t)cat.M - 1);
  hipError_t e = end_bit <= 32 ? group_nodes<uint32_t>(C, n, cat, b, sb, end_bit, s)
                               : group_nodes<uint64_t>(C, n, cat, b, sb, end_bit, s);
  if (e != hipSuccess) return e;
  // key_in and key_out are free after k_nodes; vec slot 7 is unused by the
  // solver, and slot 4 (the CG residual, written only later) holds the
  // right-hand-side terms until k_node_init has summed them
  int32_t* nbr = (int32_t*)sb.key_out;
  double* wgt = sb.vec + 7 * E;
  double* rv = sb.vec + 4 * E;
  hipLaunchKernelGGL(k_edges, dim3(grid_for(E)), dim3(kBlock), 0, s, E, sb.val_out, sb.node_of,
                     b.wr, nbr, wgt, rv);
  SolveArgs a;
  a.vals = sb.val_out;
  a.node_of = sb.node_of;
  a.nbr = nbr;
  a.wgt = wgt;
  a.node_start = sb.node_start;
  a.seg_begin = sb.seg_begin;
  a.seg_end = sb.seg_end;
  a.w = b.w;
  a.r = b.r;
  a.A = sb.vec;
  a.b = sb.vec + E;
  a.y = sb.vec + 2 * E;
  a.Wp = sb.vec + 3 * E;
  a.rr = sb.vec + 4 * E;
  a.p = sb.vec + 5 * E;
  a.ap = sb.vec + 6 * E;
  a.state = sb.ivec;
  a.nstate = sb.ivec + E;
  a.par = sb.ivec + 2 * E;
  a.core = sb.ivec + 3 * E;
  a.core2 = (int32_t*)sb.key_in;  // free after k_nodes (room for 2E entries)
  a.lambda = (cat.sigma * cat.sigma) / (cat.kappa * cat.kappa);
  a.max_rounds = kMaxRounds;
  a.n_entries = (int32_t)E;
  // CG to a relative residual of 1e-16 (z = (r - U y)/sigma^2 scales y
  // errors by 1/sigma^2, so y is solved to FP64 rounding), at most 1,000
  // iterations per pass and three passes; a core still above 1e-8 after them
  // is an error
  a.max_iter = 1000;
  a.tol2 = 1e-32;
  a.accept2 = 1e-16;
  a.err = err;
  // nodes: at most one per entry; the kernels stop at the node count on the device
  hipLaunchKernelGGL(k_node_init, dim3(grid_for(E)), dim3(kBlock), 0, s, sb.count, a.node_start,
                     wgt, rv, a.lambda, a.A, a.b, a.state, a.par);
  hipLaunchKernelGGL(k_pairs, dim3(grid_for(E)), dim3(kBlock), 0, s, sb.count, a.node_start, a.nbr,
                     a.wgt, a.A, a.b, a.y, a.state);
  hipLaunchKernelGGL(k_tree_solve<kTreeBlock>, dim3((unsigned)(C * cat.L)), dim3(kTreeBlock), 0, s, a);
  hipLaunchKernelGGL(k_exact_z, dim3(grid_for((int64_t)C * n)), dim3(kBlock), 0, s,
                     (int64_t)C * n, cat.sigma * cat.sigma, b.w, b.r, sb.node_of, a.y, b.sta,
                     cat.L_p, cat.zscale_s, b.z);
  return hipGetLastError();
}

// Entries sorted by (chain, event) with K-bit keys; the first entry of each
// run sums the run in entry order into G[chain][event].
template <class K>
hipError_t event_runs(int C, int64_t n, const CatView& cat, double scale, const BatchBufs& b,
                      const SortBufs& sb, double* G, int end_bit, hipStream_t s) {
  const int64_t E = 2 * (int64_t)C * n;
  K* key_in = (K*)sb.key_in;
  K* key_out = (K*)sb.key_out;
  hipLaunchKernelGGL(k_event_keys<K>, dim3(grid_for(E)), dim3(kBlock), 0, s, C, n, cat.M, b,
                     key_in, sb.val_in);
  size_t tb = sb.temp_bytes;
  hipError_t e = rocprim::radix_sort_pairs(sb.temp, tb, key_in, key_out, sb.val_in, sb.val_out,
                                           (size_t)E, 0, end_bit, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)C * cat.M * 4)), dim3(kBlock), 0, s, G, 0.0,
                     (int64_t)C * cat.M * 4);
  hipLaunchKernelGGL(k_reduce_runs<K>, dim3(grid_for(E)), dim3(kBlock), 0, s, key_out,
                     sb.val_out, E, scale, b, G);
  return hipGetLastError();
}

hipError_t reduce_events(const CatView& cat, int C, int64_t n, double scale, BatchBufs b,
                         SortBufs sb, double* G, hipStream_t s) {
  const int end_bit = bits_for((uint64_t)C * (uint64_t)cat.M - 1);
  return end_bit <= 32 ? event_runs<uint32_t>(C, n, cat, scale, b, sb, G, end_bit, s)
                       : event_runs<uint64_t>(C, n, cat, scale, b, sb, G, end_bit, s);
}

void launch_centroid(const double* theta, int C, int M, double* partial, double* thetabar,
                     hipStream_t s) {
  const int nchunk = (int)ceil_div(M, kCentroidChunk);
  hipLaunchKernelGGL(k_centroid_partial, dim3(nchunk, C), dim3(kBlock), 0, s, theta, M, nchunk,
                     partial);
  hipLaunchKernelGGL(k_centroid_final, dim3(C), dim3(64), 0, s, partial, nchunk, M, thetabar);
}

void launch_update(const CatView& cat, int C, double* theta, double* v, const double* G,
                   const double* thetabar, int64_t* steps, int64_t* mcount, const UpdateArgs& a,
                   double* mean, double* m2, hipStream_t s) {
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
  hipLaunchKernelGGL(k_advance, dim3(grid_for(C, 64)), dim3(64), 0, s, C, steps, mcount, a.burn,
                     a.thin);
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

void launch_batch_terms_out(int64_t n, const BatchBufs& b, double* T_i, double* T_j, double* gT_i,
                            double* gT_j, double* r, double* z, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_terms_out, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b, T_i, T_j,
                     gT_i, gT_j, r, z);
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

void launch_linear_keep(const BatchBufs& b, const double* theta, int64_t n, double e_max,
                        uint8_t* keep, unsigned long long* count, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_linear_keep, dim3(grid_for(n)), dim3(kBlock), 0, s, b, theta, n, e_max,
                     keep, count);
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
