/*
 * spider.h - C ABI of libspider, the MI355X (gfx950) hot path of SPIDER,
 * "Scalable Probabilistic Inference for Differential Earthquake Relocation"
 * (Ross, Wilding, Azizzadenesheli, Kato; arXiv 2508.12117).
 *
 * One step of the path, for every chain of a catalog:
 *   minibatch of n double-difference observations (Sec. 3.2, N/n batches
 *   per epoch) -> travel times T(x; s) and source gradients from a neural
 *   travel-time network (Sec. 3.2, EikoNet; any differentiable T, Sec. 5) ->
 *   residuals r = tau - [T(x_i;s) - T(x_j;s) + t_i - t_j] (Eq. 1,
 *   eq:forwardmodel) -> whitening z = Sigma_B^{-1} r with the marginal
 *   covariance of eq:marginal_sigma and the weights of eq:correlation_decay
 *   (Sec. 3.1) -> per-event gradient of the 4 parameters (x, y, z, t), scaled
 *   by N/n (eq:sgd) plus event and centroid priors (Sec. 3.1) -> SGLD or
 *   pSGLD update with Gaussian noise (Sec. 3.2, eq:pSGLD) -> per-event
 *   posterior mean and covariance (Sec. 3.4).
 *
 * Conventions (all entry points):
 *  - Return value: SPIDER_OK (0) or a negative SPIDER_E_* code.  Nothing
 *    aborts or throws across the ABI; spider_last_error() explains the last
 *    failure of a context.
 *  - A context is bound to one device and one HIP stream and is not
 *    thread-safe.  All device work is enqueued on that stream; entry points
 *    return without waiting unless stated otherwise.
 *  - Input arrays stay owned by the caller and are copied at load.  Output
 *    arrays are allocated by the caller on the context's device ("device
 *    pointer" below); the library owns only its internal device memory and
 *    frees it in spider_destroy().
 *  - Units: km and s; z is depth (positive down); stations have z = 0 in the
 *    shipped workloads but any z is accepted.
 *  - Row-major layouts throughout: [M][4] means 4 consecutive doubles
 *    (x, y, z, t) per event.
 */
#ifndef SPIDER_H
#define SPIDER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SPIDER_OK = 0,
  SPIDER_E_INVALID = -1,     /* bad argument, id or input value */
  SPIDER_E_OOM = -2,         /* device allocation failed */
  SPIDER_E_HIP = -3,         /* HIP runtime error */
  SPIDER_E_STATE = -4,       /* call not valid in the current state */
  SPIDER_E_UNSUPPORTED = -5, /* valid but not supported by this build */
  SPIDER_E_NUMERIC = -6      /* non-finite state after an update */
};

enum { SPIDER_MEM_HOST = 0, SPIDER_MEM_DEVICE = 1 };
/* Whitening of the minibatch residuals (Sec. 3.1):
 *   NONE  z = r / sigma^2                                  (kappa ignored)
 *   DIAG  z = r / (sigma^2 + 2 kappa^2 w)   (diagonal of Sigma_B only)
 *   EXACT z = Sigma_B^{-1} r, Sigma_B = sigma^2 I + kappa^2 W^{1/2} A A^T W^{1/2}
 *         restricted to the batch's observations of each group          */
enum { SPIDER_WHITEN_NONE = 0, SPIDER_WHITEN_DIAG = 1, SPIDER_WHITEN_EXACT = 2 };
/* Arithmetic of the network's hidden layers: FP32, or BF16 MFMA operands
 * with FP32 accumulation.  Inputs, first and output layers, travel-time
 * assembly, residuals, whitening, gradient and state are FP32/FP64 in both. */
enum { SPIDER_FP32 = 0, SPIDER_BF16 = 1 };
/* spider_grad flags */
enum { SPIDER_GRAD_PRIOR = 1, SPIDER_GRAD_CENTROID = 2, SPIDER_GRAD_L1 = 4 };

#define SPIDER_MAX_LAYERS 16

typedef struct spider_ctx spider_ctx;

/* Library version (major * 10000 + minor * 100 + patch). */
int spider_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *ctx receives the
 * handle.  Errors: SPIDER_E_INVALID (no such device), SPIDER_E_HIP. */
int spider_create(spider_ctx** ctx, int device, void* hip_stream);

/* Wait for the context's stream and free everything it owns.  NULL is a no-op. */
void spider_destroy(spider_ctx* ctx);

/* Text of the last error on this context; owned by the context, valid until
 * its next call.  Never NULL. */
const char* spider_last_error(const spider_ctx* ctx);

/* Block until all work enqueued by this context has finished.
 * Errors: SPIDER_E_HIP with the runtime's message. */
int spider_sync(spider_ctx* ctx);

/* ---- catalog (Sec. 3.1: M events, L stations, dd observations) --------- */
typedef struct {
  int32_t M;                /* events, >= 2                                    */
  int32_t L;                /* stations, >= 1; the group g of an observation is
                               its station + L * phase (Sec. 3.1)            */
  int32_t P;                /* event pairs, >= 1                              */
  int64_t N;                /* observations, >= 1                             */
  int32_t mem;              /* SPIDER_MEM_HOST or _DEVICE for every array     */
  const double* hypo0;      /* [M][4] initial hypocentre and origin time; also
                               the event-prior mean mu_e (Sec. 3.1)           */
  const double* stations;   /* [L][3] station coordinates                     */
  const int32_t* pair_i;    /* [P] first event xi^1 of each pair, in [0, M)   */
  const int32_t* pair_j;    /* [P] second event xi^2, in [0, M), != pair_i    */
  const int32_t* obs_pair;  /* [N] pair of each observation, in [0, P)        */
  const int16_t* obs_sta;   /* [N] station of each observation, in [0, L)     */
  const float* obs_dt;      /* [N] observed differential time tau_n (s)       */
  double sigma;             /* IID noise s.d. sigma_P (s), > 0                */
  double kappa;             /* shared-event s.d. kappa_P (s), >= 0            */
  double p;                 /* weight decay exponent p (eq:correlation_decay) */
  double ell;               /* weight length scale ell (km), > 0              */
  double eps_w;             /* weight floor epsilon, > 0                      */
  double prior_sigma[4];    /* event prior s.d. (x, y, z km; t s), > 0        */
  double centroid_sigma[4]; /* centroid prior s.d., > 0                       */
  uint32_t stream;          /* random-stream id of this catalog, < 2^24       */
  int32_t whiten;           /* SPIDER_WHITEN_*                                */
  const int8_t* obs_phase;  /* [N] phase of each observation, 0 = P, 1 = S, or
                               NULL for all P.  A catalog with S observations
                               has 2L groups and needs an S network
                               (spider_set_phase_net)                          */
  double sigma_s;           /* S-phase sigma_S (s), > 0 (two phases only)      */
  double kappa_s;           /* S-phase kappa_S (s), >= 0, and > 0 exactly when
                               kappa > 0 (two phases only)                     */
} spider_catalog_desc;

/* Load a catalog (Sec. 3.1).  Copies every array to the device, then on the
 * device: edge weights w~_e = (d_e/ell)^p + eps_w with d_e = |x_i - x_j| at
 * the initial locations (eq:correlation_decay), normalised to mean 1 over
 * each group's observations; the centroid prior mean mu_c = mean of hypo0.
 * Errors: SPIDER_E_INVALID for out-of-range ids, i == j, non-finite values,
 * non-positive sigma/ell/eps_w/prior s.d., an observation whose initial
 * source lies within 1e-3 km of its station; SPIDER_E_UNSUPPORTED for more
 * than 40,960 station-phase groups; SPIDER_E_OOM; SPIDER_E_HIP.
 * Synchronous (the arrays may be reused when it returns). */
int spider_load_catalog(spider_ctx* ctx, const spider_catalog_desc* desc, int32_t* cat_id);

/* The S-phase travel-time network of a two-phase catalog (Sec. 3.1: one
 * forward model per phase): every later call that evaluates the catalog's
 * observations runs its S rows through `net_id` and its P rows through the
 * network the call names, in the call's precision.  Two-phase catalogs are
 * stepped one chain set at a time (never fused with other catalogs), and
 * each minibatch waits once for the count of its P rows.  Calls on a
 * two-phase catalog without one fail with SPIDER_E_STATE.
 * Errors: SPIDER_E_INVALID (ids). */
int spider_set_phase_net(spider_ctx* ctx, int32_t cat_id, int32_t net_id);

/* ---- travel-time network (Sec. 3.2: EikoNet; Sec. 5: any differentiable T)
 * u = ((x - center)/half_extent, (s - center)/half_extent)   (6 inputs)
 * a_1 = tanh(W[0] u + b[0]); a_{l+1} = tanh(W[l] a_l + b[l]), l = 1..D-1
 * o = W[D] a_D + b[D];  T = |x - s| / v0 * softplus(o) / ln 2              */
typedef struct {
  int32_t D;                /* hidden tanh layers, 1..SPIDER_MAX_LAYERS       */
  int32_t H;                /* hidden width, a multiple of 16, 16..256        */
  int32_t mem;              /* SPIDER_MEM_HOST or _DEVICE for W and b         */
  const float* W[SPIDER_MAX_LAYERS + 1]; /* W[0]: [H][6]; W[1..D-1]: [H][H];
                                            W[D]: [H] (output row), row-major */
  const float* b[SPIDER_MAX_LAYERS + 1]; /* b[0..D-1]: [H]; b[D]: [1]        */
  double v0;                /* scale speed (km/s), > 0                        */
  double center[3];         /* input centre c0                                */
  double half_extent[3];    /* input half extent h, > 0                       */
} spider_net_desc;

/* Load a network: FP32 copies and the BF16 / FP32 operand packings of the
 * hidden layers for the matrix-core kernels.  Synchronous.
 * Errors: SPIDER_E_INVALID (shape or non-finite weights), SPIDER_E_OOM,
 * SPIDER_E_HIP. */
int spider_load_net(spider_ctx* ctx, const spider_net_desc* desc, int32_t* net_id);

/* T(x; s) and dT/dx for `rows` source/receiver pairs.  x_src, s: device
 * [rows][3]; T: device [rows]; gradT: device [rows][3] or NULL.  One kernel
 * runs the forward pass and then the reverse-mode source gradient (Sec. 3.2):
 * the derivative factors 1 - a^2 of the hidden layers stay in registers and
 * LDS between the two passes, so no activation is written to memory and
 * nothing is recomputed.  rows may be 0.
 * Errors: SPIDER_E_INVALID (ids, rows < 0, NULL required pointers). */
int spider_travel_time(spider_ctx* ctx, int32_t net_id, int32_t precision,
                       const double* x_src, const double* s, int64_t rows,
                       double* T, double* gradT);

/* The two halves of a differentiable T (Sec. 3.2 and Sec. 5: any
 * differentiable travel-time model), for a reverse-mode caller such as an
 * autograd engine.  spider_tt_forward writes T only (device [rows]).
 * spider_tt_backward evaluates the network again at the same points (the
 * activations of the forward call are not kept anywhere) and writes the
 * vector-Jacobian product grad_x[r] = grad_T[r] dT/dx(x_src[r]; s[r])
 * (device [rows][3]) for the source only; grad_T is device [rows].
 * x_src, s: device [rows][3].  rows may be 0.
 * Errors: SPIDER_E_INVALID (ids, rows < 0, NULL pointers). */
int spider_tt_forward(spider_ctx* ctx, int32_t net_id, int32_t precision,
                      const double* x_src, const double* s, int64_t rows, double* T);
int spider_tt_backward(spider_ctx* ctx, int32_t net_id, int32_t precision,
                       const double* x_src, const double* s, const double* grad_T,
                       int64_t rows, double* grad_x);

/* ---- allocation-free travel time ----------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * spider_travel_time with the same arguments, results and errors, whose
 * scratch (the network kernel's per-row outputs) is a fixed array compiled
 * into the library instead of the context's workspace.  Each device the
 * library runs on holds its own copy of that array (16 MiB) until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and never tunes or profiles the network launch:
 * it uses the context's tuned tile variant if there is one (every variant
 * gives the same bits).  rows <= SPIDER_NOALLOC_MAX_ROWS, else
 * SPIDER_E_INVALID.  All calls on one device share its array: calls that
 * overlap on one GPU (several streams or contexts) race, and the caller
 * must order them. */
#define SPIDER_NOALLOC_MAX_ROWS 1048576
int spider_travel_time_noalloc(spider_ctx* ctx, int32_t net_id, int32_t precision,
                               const double* x_src, const double* s, int64_t rows,
                               double* T, double* gradT);

/* ---- one stochastic gradient (eq:sgd) ----------------------------------
 * g = [prior terms] + (N/n) * sum_{k<n} (d tau^_k / d theta)^T z_k
 * at state theta (device [M][4]).  The batch is batch_idx (device [n]
 * observation indices in [0, N), repeats allowed) or, if batch_idx is NULL,
 * minibatch `step` of chain `chain` under `seed` (see spider_batch_indices).
 * flags: SPIDER_GRAD_PRIOR adds -(theta - hypo0)/prior_sigma^2,
 * SPIDER_GRAD_CENTROID adds -(mean(theta) - mu_c)/(M centroid_sigma^2) to
 * every event (Sec. 3.1).  SPIDER_GRAD_L1 replaces the likelihood term by
 * the negative gradient of the Stage 1 loss (eq:stage1loss with the L1
 * norm, Sec. 3.2), L = (1/n) sum_{k<n} |r_k|: (1/n) sum_k sign(r_k)
 * (d tau^_k / d theta), and logpost_out then holds -L + log priors.
 * grad_out: device [M][4] (events outside the batch get only the prior
 * terms).  logpost_out: device [1] or NULL: -(N/n)/2 r^T z + log priors, up
 * to an additive constant.  Errors: SPIDER_E_INVALID (ids, n < 1, n > N
 * without batch_idx, unknown flags). */
int spider_grad(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                const double* theta, const int64_t* batch_idx, int64_t n,
                uint64_t seed, int32_t chain, int64_t step, uint32_t flags,
                double* grad_out, double* logpost_out);

/* Per-observation terms of one minibatch, for checking each stage: travel
 * times T_i, T_j [n], source gradients gT_i, gT_j [n][3], residuals r [n]
 * and whitened residuals z [n] (device pointers, each may be NULL).
 * Arguments as spider_grad.  Errors: as spider_grad. */
int spider_batch_terms(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                       const double* theta, const int64_t* batch_idx, int64_t n,
                       uint64_t seed, int32_t chain, int64_t step,
                       double* T_i, double* T_j, double* gT_i, double* gT_j,
                       double* r, double* z);

/* Observation indices of minibatch `step` of chain `chain` (Sec. 3.2:
 * without replacement, N/n minibatches per epoch): epoch e = step / B,
 * batch b = step % B, B = floor(N/n); slot k holds pi(b n + k) where pi is
 * a four-round Feistel bijection of [0, N) keyed by (seed, catalog stream,
 * chain, e) with Philox4x32-10 round functions and cycle walking.
 * idx_out: device [n] int64.  Errors: SPIDER_E_INVALID (n < 1 or n > N). */
int spider_batch_indices(spider_ctx* ctx, int32_t cat_id, uint64_t seed, int32_t chain,
                         int64_t step, int64_t n, int64_t* idx_out);

/* The Langevin noise eta ~ N(0, 1) (Sec. 3.2) of step `step` of chain
 * `chain`: Philox4x32-10 keyed by seed, two blocks per event, 52-bit
 * uniforms, Box-Muller.  eta_out: device [M][4]. */
int spider_noise(spider_ctx* ctx, int32_t cat_id, uint64_t seed, int32_t chain,
                 int64_t step, double* eta_out);

/* ---- chains and the sampler (Sec. 3.2, eq:pSGLD) ------------------------ */

/* (Re)create `n_chains` chains of a catalog: theta = hypo0, v = 0, step 0,
 * empty moments (Sec. 3.2 starts from the initial locations).
 * Errors: SPIDER_E_INVALID, SPIDER_E_OOM. */
int spider_reset_chains(spider_ctx* ctx, int32_t cat_id, int32_t n_chains);

typedef struct {
  int32_t cat_id;
  int32_t net_id;
  int32_t n_chains;         /* chains 0..n_chains-1 of the catalog advance    */
  int32_t precision;        /* SPIDER_FP32 or SPIDER_BF16                     */
  int64_t batch;            /* minibatch size n per chain, 1..N               */
} spider_chainset;

typedef struct {
  double step;              /* epsilon_t (fixed)                              */
  double beta2;             /* pSGLD second-moment decay, in [0, 1]           */
  double eps_p;             /* pSGLD epsilon in V = 1/(sqrt(v) + eps_p), > 0  */
  double noise_scale;       /* a: multiplies the injected noise (1 sampling,
                               0 noise off: the warm-up stage of Sec. 3.2),
                               >= 0                                           */
  int32_t precond;          /* 0: SGLD  theta += eps g + a sqrt(2 eps) eta
                               1: pSGLD v = b2 v + (1-b2) g*g;
                                  V = 1/(sqrt(v)+eps_p);
                                  theta += eps V g + a sqrt(2 eps V) eta      */
  int32_t noise_ramp;       /* 0: a = noise_scale at every step of the call;
                               1: a rises linearly over the call (the ramp
                               stage of Sec. 3.2): step k = 0 .. n_steps-1
                               of the call uses a = noise_scale +
                               (noise_scale_end - noise_scale) k / n_steps    */
  int64_t n_steps;          /* steps to run, >= 0                             */
  int64_t burn_in;          /* after the update of global step t, theta enters
                               the moments iff t >= burn_in and
                               (t - burn_in) % thin == 0                      */
  int64_t thin;             /* >= 1                                           */
  uint64_t seed;            /* keys the batch and noise streams               */
  double noise_scale_end;   /* with noise_ramp = 1: the amplitude the ramp
                               reaches after the call, >= 0                   */
} spider_sgld_cfg;

/* Advance every chain of every set by cfg->n_steps steps.  Each step uses
 * the chain's global step counter for its batch and noise, so a run split
 * over calls equals one uninterrupted run (a ramp of the noise amplitude
 * is defined per call, so a split ramp passes the matching amplitudes to
 * each part).  The paper's schedule after its first stage is three calls:
 * warm-up with noise_scale 0, the ramp 0 -> 1, then sampling with
 * noise_scale 1 and burn_in at the first sampling step.  Chains are created
 * on first use
 * if the catalog has fewer.  After the last step every state is checked for
 * finite values: SPIDER_E_NUMERIC names the catalog and chain otherwise
 * (this waits for the stream).  When there are several sets, all with the
 * same network and precision and no catalog twice, they advance in fused
 * steps: one network launch per step evaluates the rows of every set, and
 * the results equal those of advancing each set on its own.  Errors:
 * SPIDER_E_INVALID, SPIDER_E_NUMERIC, SPIDER_E_OOM, SPIDER_E_HIP. */
int spider_sgld_steps(spider_ctx* ctx, const spider_chainset* sets, int32_t n_sets,
                      const spider_sgld_cfg* cfg);

/* HIP graphs for spider_sgld_steps (default on).  When a call's sets advance
 * in fused steps, the noise amplitude is constant over the call and
 * profiling is off, the first step runs eagerly and the others are replayed
 * from a HIP graph of one step captured on a private stream of the context
 * (every kernel reads the chains' step counters on the device, so each
 * replay is the next step; the results equal those of launching every step,
 * bit for bit).  enable = 0 launches every step on the stream.
 * Errors: SPIDER_E_INVALID (null context). */
int spider_set_graphs(spider_ctx* ctx, int enable);

/* ---- Stage 1: a robust initial solution (Sec. 3.2, eq:stage1loss) -----
 * Minimises the L1 loss of the dd residuals, L = (1/n) sum_{k<n} |r_k| over
 * each chain's minibatch, with Adam and no priors, starting from the chains'
 * current states.  Step t of chain c uses the sampler's minibatch of (seed,
 * catalog stream, c, t) and the bias correction of Adam step k = t + 1 (t =
 * the chain's step counter): with g = -(1/n) sum_k sign(r_k) dtau^_k/dtheta,
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
 * m and v start at zero after spider_reset_chains; the step counters
 * advance (the sampler stages continue the same minibatch stream) and no
 * moments are recorded.  Non-finite states are reported as by
 * spider_sgld_steps.  Errors: SPIDER_E_INVALID, SPIDER_E_NUMERIC,
 * SPIDER_E_OOM, SPIDER_E_HIP. */
typedef struct {
  double lr;                /* Adam learning rate (Table 1: 1e-3, 1e-4), > 0  */
  double beta1;             /* first-moment decay, in [0, 1) (0.9)            */
  double beta2;             /* second-moment decay, in [0, 1) (0.999)         */
  double eps;               /* > 0 (1e-8)                                     */
  int64_t n_steps;          /* steps to run, >= 0                             */
  uint64_t seed;            /* keys the batch stream                          */
} spider_map_cfg;
int spider_map_steps(spider_ctx* ctx, const spider_chainset* sets, int32_t n_sets,
                     const spider_map_cfg* cfg);

/* Outlier screening after Stage 1 (Sec. 3.2): the residuals r of all N
 * observations at chain `chain`'s state (the network in `precision`), their
 * median and median absolute deviation MAD = median |r - median(r)| (the
 * mean of the middle two values for an even count), and keep[i] = 1 iff
 * |r_i - median(r)| <= k_mad MAD (the paper uses k_mad = 4), else 0.  The
 * caller loads the kept observations as a new catalog (its edge weights are
 * then normalised over them).  keep: device [N] uint8, caller-allocated;
 * n_keep, median, mad: host, each may be NULL.  Synchronous; allocates
 * scratch for three N-double arrays.  Errors: SPIDER_E_INVALID (ids,
 * chain, k_mad <= 0, NULL keep), SPIDER_E_OOM, SPIDER_E_HIP. */
int spider_outliers(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                    int32_t chain, double k_mad, uint8_t* keep, int64_t* n_keep, double* median,
                    double* mad);

/* Linear-regime data filter (Sec. 2.1, eq:dd_linearization; 5% in Sec. 4):
 * for every observation of pair (i, j) at station s, at chain `chain`'s state
 * and with the network in `precision`, dT = T(x_j; s) - T(x_i; s) and its
 * first-order expansion lin = grad_x T(x_i; s) . (x_j - x_i); keep[q] = 1
 * iff |dT - lin| <= max_rel_err |dT| (the paper uses 0.05), else 0.  Run it
 * at the initial locations (after spider_reset_chains) to filter the data
 * before inversion; the caller loads the kept observations as a new catalog.
 * keep: device [N] uint8, caller-allocated; n_keep: host, may be NULL.
 * Synchronous.  Errors: SPIDER_E_INVALID (ids, chain, max_rel_err < 0,
 * NULL keep), SPIDER_E_OOM, SPIDER_E_HIP. */
int spider_linearity(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                     int32_t chain, double max_rel_err, uint8_t* keep, int64_t* n_keep);

/* ---- samples and sampler diagnostics (Sec. 3.4, Sec. 3.6, Sec. 5) -------
 * Thinned samples: while a buffer is attached, every recorded state (the
 * steps that enter the moments) of chain c is also written to
 * samples[slot][C][M][4], slot = the chain's number of recorded states
 * before it (0 after spider_reset_chains), C = the catalog's chain count, as
 * long as slot < capacity.  samples: device, caller-owned and kept alive
 * while attached, room for capacity * C * M * 4 doubles; NULL detaches.
 * spider_reset_chains detaches it (attach after resetting).
 * Errors: SPIDER_E_INVALID, SPIDER_E_STATE (no chains yet). */
int spider_set_sample_buffer(spider_ctx* ctx, int32_t cat_id, double* samples,
                             int64_t capacity);

/* Percentiles of each parameter over stored samples (Sec. 3.4 credibility
 * intervals, e.g. probs 0.005 and 0.995): samples device [n_samples][n_params]
 * (a sample buffer holding K recorded states of C chains is [K * C][M * 4]);
 * out device [n_probs][n_params] receives, for each probability p, the
 * linear interpolation between the order statistics around (n_samples - 1)
 * p.  probs: host [n_probs], each in [0, 1].  n_samples <= 8192.
 * Synchronous.  Errors: SPIDER_E_INVALID, SPIDER_E_UNSUPPORTED. */
int spider_quantiles(spider_ctx* ctx, const double* samples, int64_t n_samples, int64_t n_params,
                     const double* probs, int32_t n_probs, double* out);

/* Calibration against a known truth (Sec. 4 synthetic test): frac[p] =
 * (#{samples < values[p]} + #{samples == values[p]} / 2) / n_samples, the
 * position of values[p] among parameter p's samples.  samples device
 * [n_samples][n_params]; values, frac device [n_params].  Enqueued.
 * Errors: SPIDER_E_INVALID. */
int spider_sample_ranks(spider_ctx* ctx, const double* samples, int64_t n_samples,
                        int64_t n_params, const double* values, double* frac);

/* Effective sample size (Sec. 5) of each parameter over draws
 * samples[n_draws][n_chains][n_params] (a sample buffer's layout): within-
 * chain variance W (divisor n_draws - 1), between-chain variance of the
 * chain means, var+ = (K - 1)/K W + B/K, lag-t autocorrelations
 * rho_t = 1 - (W - mean over chains of the lag-t autocovariance, divisor K)
 * / var+, rho_0 = 1, Geyer's initial positive and monotone sequence over
 * the pair sums rho_2k + rho_2k+1, tau = -1 + 2 sum, ESS = n_chains K / tau
 * (NaN for constant draws).  ess: device [n_params].  n_draws >= 4,
 * n_chains <= 64.  Enqueued.  Errors: SPIDER_E_INVALID, SPIDER_E_UNSUPPORTED. */
int spider_ess(spider_ctx* ctx, const double* samples, int64_t n_draws, int32_t n_chains,
               int64_t n_params, double* ess);

/* Step-size diagnostic (Sec. 3.6, Sec. 5): at chain `chain`'s current state,
 * the likelihood gradients of its next n_batches sampler minibatches (steps
 * t, t+1, ... of its counter, cfg->seed, `batch` observations each), their
 * per-coordinate variance Var(g) (divisor n_batches - 1), and ratio[m][k] =
 * step V Var(g) / (2 noise_scale^2): the variance of the drift step V g over
 * that of the injected noise, with V = 1/(sqrt(v) + eps_p) from the chain's
 * preconditioner (cfg->precond = 1) or 1.  The paper targets 0.1-1.0.
 * ratio: device [M][4]; *mean_ratio (host, may be NULL) their mean.  Uses
 * step, eps_p, noise_scale, precond and seed of cfg; the chain is not
 * advanced.  Synchronous.  Errors: SPIDER_E_INVALID, SPIDER_E_HIP. */
int spider_noise_ratio(spider_ctx* ctx, int32_t cat_id, int32_t net_id, int32_t precision,
                       int32_t chain, int64_t batch, int32_t n_batches, const spider_sgld_cfg* cfg,
                       double* ratio, double* mean_ratio);

/* Posterior moments (Sec. 3.4) of a catalog: chain >= 0 for one chain, -1
 * for all chains pooled (pairwise combination of Chan, Golub and LeVeque).
 * mean: device [M][4]; cov: device [M][10] upper triangle xx xy xz xt yy yz
 * yt zz zt tt with divisor count - 1 (either may be NULL); *count (host)
 * receives the number of samples.  Enqueued on the stream.
 * Errors: SPIDER_E_INVALID, SPIDER_E_STATE (no chains). */
int spider_moments(spider_ctx* ctx, int32_t cat_id, int32_t chain,
                   double* mean, double* cov, int64_t* count);

/* Copy a chain's state out (theta, v: device [M][4], either may be NULL) and
 * its global step counter (*step, host, may be NULL). */
int spider_get_state(spider_ctx* ctx, int32_t cat_id, int32_t chain,
                     double* theta, double* v, int64_t* step);

/* Overwrite a chain's state (theta, v: device [M][4], v may be NULL for 0)
 * and step counter; the moments are left as they are. */
int spider_set_state(spider_ctx* ctx, int32_t cat_id, int32_t chain,
                     const double* theta, const double* v, int64_t step);

/* ---- measurement --------------------------------------------------------
 * While enabled, every launch of the travel-time network kernel made by this
 * context is bracketed by HIP events recorded on the context's stream.
 * spider_profile(ctx, 1) enables and clears the record, 0 disables it.
 * spider_profile_read waits for the stream and returns the summed kernel
 * time (ms), the number of launches and the network rows they processed
 * (each pointer may be NULL).  Errors: SPIDER_E_INVALID, SPIDER_E_HIP. */
int spider_profile(spider_ctx* ctx, int enable);
/* Tile shape of the matrix-core network kernel this context uses for a
 * network and precision: *waves per workgroup, *row_tiles of 16 rows per
 * workgroup and *schedule (0: one workgroup barrier per layer, 1: row halves
 * in ping-pong with a weight ring of one layer, 2: the same with one and a
 * half layers); 0, 0, 0 when the shape has no matrix-core kernel.  The
 * variant is chosen by timing every compiled one on the first launch of at
 * least 65,536 rows (all variants give identical results).  Any output
 * pointer may be NULL.  Errors: SPIDER_E_INVALID (unknown network id). */
int spider_network_variant(spider_ctx* ctx, int32_t net_id, int32_t precision, int32_t* waves,
                           int32_t* row_tiles, int32_t* schedule);
int spider_profile_read(spider_ctx* ctx, double* ms, int64_t* launches, int64_t* rows);

#ifdef __cplusplus
}
#endif

#endif /* SPIDER_H */
