// Internal declarations of libspider shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "net_rows.h"

namespace spider {

// One observation record as loaded: 12 bytes, loaded as three dwords.
struct Obs {
  int32_t pair;
  float dt;
  int32_t sta;
};

// What the minibatch gather reads of an observation, packed once at load
// into one aligned 32-byte record (a single cache line per random read):
// the pair's events, the group, tau and the normalised edge weight
// w = w~_pair * inv_mean[group].
struct __attribute__((aligned(32))) ObsRec {
  int32_t i, j, g;
  float dt;
  double w;
  double pad;
};

// Catalog as the step kernels see it.
struct CatView {
  int32_t M, L;
  int64_t N;
  const double* hypo0;     // [M][4]
  const double* stations;  // [L][3]
  const int2* pairs;       // [P] (i, j)
  const double* w_pair;    // [P] unnormalised edge weight
  const ObsRec* rec;       // [N] packed observation records
  const double* inv_mean;  // [L] 1 / group mean of the edge weights
  const double* mu_c;      // [4] centroid prior mean
  uint32_t stream;
  double sigma, kappa;
  // Two-phase catalogs: groups g >= L_p are S groups (L_p = L otherwise);
  // their edge weights carry the factor that maps Sigma_g onto the P
  // phase's sigma and kappa, and their z is multiplied by zscale_s.
  int32_t L_p;
  double zscale_s;
  double prior_sigma[4], centroid_sigma[4];
};

// Minibatch buffers of one chain set, C chains x n slots.  Slot q = c n + k;
// entry e = 2q is event i of the slot and e = 2q + 1 event j (E = 2 C n
// entries).  The entries are also held in CSR order: grouped by (chain,
// event) key c M + m, and inside each event's segment by (group, entry), so
// that the entries of one (chain, group, event) node of the whitening are
// contiguous and every sum over a segment or a node runs in a fixed order.
// One observation of the exact whitening as its solver gathers it, in one
// 32-byte record: weight, residual and the first CSR positions of the nodes
// of its two entries.
struct WRec {
  double w;
  double r;
  int32_t hi;
  int32_t hj;
  int32_t pad[2];
};

// Per entry, written in one 16-byte store by the assembly (entry order): the
// travel time plus the event's origin time, the entry's CSR position (bit
// 31: its node holds this entry only) and its node's first CSR position.
struct TRec {
  double T;
  int32_t p;
  int32_t head;
};

struct BatchBufs {
  int64_t* obs;     // [C n] observation index (null: not kept)
  int32_t* ev;      // [E] event of each entry
  int32_t* sta;     // [E] group of each entry (station + L_p phase)
  double* tau;      // [C n] observed differential time
  double* w;        // [C n] normalised edge weight
  int32_t* start;   // [C M + 1] first CSR position of each (chain, event) key
  int32_t* csr;     // [E] entry at each CSR position
  uint64_t* ckey;   // [E] bucket records (event in bucket, group, entry) of the CSR build
  int32_t* hd;      // [E] per CSR position: the first position of its node; bit 31: the
                    //     node has this entry only
  int32_t* pev;     // [E] event at each CSR position
  int32_t* pgr;     // [E] group at each CSR position
  int32_t* nend;    // [E] at a node's first position: one past its last
  int32_t* rows;    // [E] network row order of two-phase catalogs (CSR positions, P first)
  double* zp;       // [E] whitened residual of each CSR position's observation, negated at
                    //     the observation's second entry (event j)
  RowOut* net_out;  // [E] network output of each row
  TRec* tr;         // [E] per entry: T(x; s) + t, its CSR position, its node's first one
  float* gT;        // [E][3] source gradient at each CSR position (assembled in FP64, kept
                    //     in FP32 for the per-event sums, which run in FP64)
  double* gT64;     // [E][3] the same in FP64, written instead of gT for the calls that
                    //     return per-entry terms
  double* r;        // [C n] residual (null: not kept)
  double* z;        // [C n] whitened residual (filled from zp by launch_obs_z when asked)
  WRec* wr;         // [C n] per observation taken by the solver: (w, r, its two nodes)
};

// One entry of a node of the exact whitening, stored at the entry's CSR
// position: the observation's weight w, its residual r (negated at the
// observation's second entry, event j) and the first position of the node
// at the entry's other end.
struct ERec {
  double w;
  double rs;
  int32_t nbr;
  int32_t pad;
};

// A node of the exact whitening in its system's list order: the diagonal A,
// the right-hand side b, its first CSR position and its number of entries.
struct NodeRec {
  double A;
  double b;
  int32_t q;
  int32_t ne;
};

// Scratch of the exact whitening of one chain set (all arrays indexed by CSR
// position unless stated; a node is stored at its first position).
struct SolveBufs {
  int32_t* act;       // [E] 1 at the first position of every node the solver takes
  int32_t* sys;       // [C L nb + 1] nodes per (chain, group, position block), then list
                      // offsets (system s = c L + g starts at sys[s nb])
  int32_t* list;      // [E] nodes of each system (first positions)
  ERec* ent;          // [E] per position of a listed node: its observation's entry record
  double* vec;        // [7][E] A, b, y, Wp, rr, p, ap
  int32_t* ivec;      // [5][E] state, nstate, par, next list, elimination order
  int32_t* lidx;      // [E] at a node's first position: its index in its system's list
  NodeRec* nrec;      // [E] the nodes in list order (same offsets as list)
  int32_t* spill;     // [C L] 1: the system is solved from global memory (too large for LDS)
  int32_t* scan_part; // scratch of the scans
};

// Position blocks per chain of the exact whitening's system lists for
// C chains of 2n entries and L groups (at most 2^22 list counts), and the
// positions per block.
int64_t list_blocks(int64_t C, int64_t n, int64_t L);
int64_t list_block_span(int64_t n, int64_t nb);

// Exclusive prefix sum of a[0..len) in place, a[len-1] receiving the sum of
// all earlier entries (deterministic; part holds ceil(len / 4096) + 1 ints).
void launch_scan(int32_t* a, int64_t len, int32_t* part, hipStream_t s);
int64_t scan_part_size(int64_t len);

// ---- launchers (each enqueues on stream s; errors surface via hipGetLastError)
// Network kernels (mlp_*.hip).  Unsupported shapes return hipErrorNotSupported.
hipError_t launch_mlp_tangent(const RowSource& src, const NetView& net, RowOut* out,
                              hipStream_t stream);
// Matrix-core kernel variants (tile shapes) of one network shape: NW waves
// per workgroup, RT 16-row tiles per workgroup.  Every variant computes the
// same per-row arithmetic in the same order, so they agree bit for bit.
struct MlpVariant {
  int nw, rt;
  int schedule;  // 0: one barrier per layer (k_mlp), 1: row-half ping-pong (k_mlp_pp)
  hipError_t (*launch)(const RowSource&, const NetView&, RowOut*, hipStream_t);
};
// Number of variants for (precision, H, D) and the list (0: no kernel).
int mlp_variants(int precision, int H, int D, const MlpVariant** list);
int mlp_variants_bf16(int H, int D, const MlpVariant** list);
int mlp_variants_f32(int H, int D, const MlpVariant** list);
bool mlp_mfma_supported(int precision, int H, int D);
// Bytes of the forward (or backward) operand pack of one hidden layer.
size_t mfma_pack_bytes(int precision, int H);
// Packs hidden layer W (row-major [H][H] fp32, host) into the forward and
// backward matrix-core operand orders (host buffers of mfma_pack_bytes each).
void mfma_pack_layer(int precision, int H, const float* W, void* fwd, void* bwd);

// Load-time kernels (step.hip).
void launch_pair_weights(const double* hypo0, const int2* pairs, int64_t P, double ell, double p,
                         double eps_w, double* w_pair, hipStream_t s);
// rec[t] = the packed record of observation t.
void launch_pack_obs(const Obs* obs, int64_t N, const int2* pairs, const double* w_pair,
                     const double* inv_mean, ObsRec* rec, hipStream_t s);
void launch_validate(const double* hypo0, int M, const double* stations, int L, const int2* pairs,
                     int64_t P, const Obs* obs, int64_t N, int* bad, hipStream_t s);
// inv_mean[g] = count_g / sum of w~ over group g; deterministic.
hipError_t group_inverse_mean(const Obs* obs, int64_t N, int L, const double* w_pair,
                              double* inv_mean, hipStream_t s);
// out[c] = mean over rows of a [rows][4] array (c = 0..3); deterministic.
void launch_mean4(const double* a, int64_t rows, double* out, hipStream_t s);

// Error bits a step sets in its device flag (read back by the host after
// the call): a minibatch index outside [0, N) or a failed permutation walk,
// and a CG solve of a cyclic core that did not converge.
constexpr int kErrSelect = 1;
constexpr int kErrSolve = 2;

// Step kernels (batch_csr.hip).
// Minibatch of each chain: explicit indices idx (all chains) or, if idx is
// null, the Feistel minibatch of chain chain0 + c at step steps[c] +
// step_scalar (steps on the device; step_scalar alone if steps is null).
// err_flag |= kErrSelect on a failed walk or an index outside [0, N).
void launch_select(const CatView& cat, int C, int64_t n, const int64_t* idx, uint64_t seed,
                   const int64_t* steps, int64_t step_scalar, int chain0, BatchBufs b,
                   int* err_flag, hipStream_t s);
// Buckets of the CSR build for C chains of n observations over M events:
// (chain, block of 2^sb events), nb of them, counted over hb blocks of
// entries; words: ints of the count matrix and bucket bases.  ok = false
// when C M is too large for the bucket counters.
struct BucketShape {
  int sb;
  int64_t nbk, nb, hb, words;
  bool ok;
};
BucketShape bucket_shape(int64_t C, int64_t n, int64_t M);
// The CSR order of the entries (after launch_select): entries bucketed by
// (chain, event block), each bucket ordered by (event, group, entry) in LDS;
// csr, pos, pev, pgr, head, nend and start.  bucket_buf: bucket_shape's
// words ints; scan_part: scan_part_size(nb + 1) ints.
void launch_build_csr(const CatView& cat, int C, int64_t n, BatchBufs b, int32_t* bucket_buf,
                      int32_t* scan_part, hipStream_t s);
// Two-phase catalogs: b.rows = the entries in CSR order, those of P groups
// first; *n_p (device) = their number.  flags: E + 1 ints of scratch.
void launch_phase_rows(const CatView& cat, int64_t E, BatchBufs b, int32_t* flags,
                       int32_t* scan_part, int64_t* n_p, hipStream_t s);
// T and dT/dx of every entry from the network outputs (row v of the network
// is entry rows[v], or csr[v] when rows is null).
void launch_assemble(const CatView& cat, const NetView& net, const NetView& net_s, int C, int64_t n,
                     const double* theta, int64_t theta_stride, const int32_t* rows, BatchBufs b,
                     bool grad64, int32_t* act_clear, hipStream_t s);
// Residuals; z for whitening none / diag / L1 and for the observations of
// exact whitening whose two nodes have one entry each (z = r / (sigma^2 +
// 2 kappa^2 w)); the others mark their nodes in sv.act (cleared by the
// assembly, which is given it for exact whitening).
void launch_residual(const CatView& cat, int C, int64_t n, const double* theta,
                     int64_t theta_stride, int whiten, BatchBufs b, SolveBufs sv, hipStream_t s);
// Exact whitening of the marked nodes: per (chain, group) lists, elimination
// + CG solve of (lambda I + U^T U) y = U^T r, z = (r - U y)/sigma^2, which
// the solvers write to zp at both entries of each observation they take.
// err |= kErrSolve when a CG core does not converge.
hipError_t exact_whiten(const CatView& cat, int C, int64_t n, BatchBufs b, SolveBufs sv, int* err,
                        hipStream_t s);
// G_lik[c][m] = scale * sum over the entries of (chain c, event m) of
// zp (dT/dx, 1) (zp carries the entry's sign), one CSR segment each, summed in a fixed order (scans over
// waves of 64 positions, then the waves in order).
void launch_reduce(const CatView& cat, int C, int64_t n, double scale, BatchBufs b, double* G,
                   void* part, hipStream_t s);
// Scratch bytes of launch_reduce's part for E entries.
int64_t reduce_part_bytes(int64_t E);
// thetabar[c] = mean over events of theta[c] (4 values per chain).
void launch_centroid(const double* theta, int C, int M, double* partial, double* thetabar,
                     hipStream_t s);
// Residual mode of k_residual beside SPIDER_WHITEN_*: z = sign(r), the
// derivative of |r| (the L1 loss of Stage 1).
constexpr int kWhitenL1 = 3;

struct AdamArgs {
  double lr, beta1, beta2, eps;
};
// Adam step of chains 0..C-1 on the loss whose negative gradient is G, with
// bias correction at the chains' step counters + 1; then steps[c] += 1.
void launch_adam(int C, int M, double* theta, double* m, double* v, const double* G,
                 int64_t* steps, const AdamArgs& a, hipStream_t s);

struct UpdateArgs {
  double step, beta2, eps_p, noise_scale;
  int precond;
  uint64_t seed;
  int64_t burn, thin;
  // recorded states also go to samples[slot][sample_C][M][4], slot = the
  // chain's sample count before the step, while slot < sample_cap
  double* samples;
  int64_t sample_cap;
  int sample_C;
};
// Priors + Langevin update of chains 0..C-1 at their device step counters,
// Welford moments on recording steps, then steps[c] += 1 (and mcount[c] on
// recording steps).
void launch_update(const CatView& cat, int C, double* theta, double* v, const double* G,
                   const double* thetabar, int64_t* steps, int64_t* mcount, const UpdateArgs& a,
                   double* mean, double* m2, hipStream_t s, bool advance = true);
// The step counters of C chains advance by one (and the moment counters
// where the step was recorded); launch_update does this unless told not to.
void launch_advance(int C, int64_t* steps, int64_t* mcount, const UpdateArgs& a, hipStream_t s);
void launch_grad_finish(const CatView& cat, const double* theta, const double* G,
                        const double* thetabar, unsigned flags, double* grad_out, hipStream_t s);
// logpost = -scale/2 sum r z + priors (flags), deterministic; tmp >= 2 * 1024 doubles.
void launch_logpost(const CatView& cat, int64_t n, double scale, const double* r, const double* z,
                    const double* theta, const double* thetabar, unsigned flags, double* tmp,
                    double* out, hipStream_t s);
// T (may be null) and dT/dx (may be null; scaled by vjp_w[r] when vjp_w is
// not null) of explicit rows from the network outputs.
void launch_tt_assemble(const NetView& net, int64_t rows, const double* x, const double* s,
                        const RowOut* out, double* T, double* gradT, const double* vjp_w,
                        hipStream_t st);
// z[q] of the first Q observations in slot order, from zp at their first
// entries (for the calls that return or sum z per observation).
void launch_obs_z(int64_t Q, const BatchBufs& b, hipStream_t s);
// Per-slot terms of the first n slots of one chain at state theta (T
// without the origin time, gT gathered from CSR order).
void launch_batch_terms_out(int64_t n, const BatchBufs& b, const double* theta, double* T_i,
                            double* T_j, double* gT_i, double* gT_j, double* r, double* z,
                            hipStream_t s);
void launch_noise(const CatView& cat, uint64_t seed, int chain, int64_t step, double* eta,
                  hipStream_t s);
void launch_finite(const double* a, int64_t count, int64_t per_chain, int* bad_chain,
                   hipStream_t s);
void launch_pool_moments(int C, int M, const double* mean, const double* m2, const int64_t* cnt,
                         double* out_mean, double* out_cov, hipStream_t s);
void launch_fill(double* p, double v, int64_t count, hipStream_t s);
// Outlier screening: idx[t] = start + t; d = |r - med|; keep = |r - med| <=
// thr with the kept count added to *count; ascending sort of N doubles
// (temp = nullptr queries *temp_bytes).
void launch_iota(int64_t* idx, int64_t start, int64_t len, hipStream_t s);
void launch_absdev(const double* r, int64_t N, double med, double* d, hipStream_t s);
void launch_keep(const double* r, int64_t N, double med, double thr, uint8_t* keep,
                 unsigned long long* count, hipStream_t s);
// Linear-regime screening of one chain's batch: keep[q] = |dT - lin| <= e_max
// |dT| with dT = T_j - T_i and lin = grad T(x_i) . (x_j - x_i).
void launch_linear_keep(const BatchBufs& b, const double* theta, int64_t n, double e_max,
                        uint8_t* keep, unsigned long long* count, hipStream_t s);
// Diagnostics over stored samples [S][P] (sample-major).
constexpr int kMaxEssChains = 64;
constexpr int64_t kMaxQuantileSamples = 8192;
hipError_t launch_quantiles(const double* samples, int64_t S, int64_t P, const double* probs,
                            int n_probs, double* out, hipStream_t s);
hipError_t launch_ranks(const double* samples, int64_t S, int64_t P, const double* values,
                        double* frac, hipStream_t s);
hipError_t launch_ess(const double* x, int64_t K, int C, int64_t P, double* ess, hipStream_t s);
void launch_welford(const double* g, int64_t n, int64_t k, double* mean, double* m2,
                    hipStream_t s);
int64_t noise_ratio_blocks(int64_t n);
void launch_noise_ratio(const double* m2, int64_t n, int64_t K, const double* v, int precond,
                        double eps_p, double step, double amp, double* ratio, double* part,
                        hipStream_t s);
hipError_t sort_doubles(const double* in, double* out, int64_t N, void* temp, size_t* temp_bytes,
                        hipStream_t s);

}  // namespace spider
