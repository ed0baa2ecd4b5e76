/*
 * pf.h -- C ABI of the MI355X (gfx950) independent-ensemble particle filter.
 *
 * The library runs M fully independent bootstrap particle filters of N
 * particles each (Crisan, Miguez, Rios, arXiv 1407.8071, Sec. 3.1 and
 * Definition 3) through one observation interval per call, entirely in
 * hand-written HIP kernels, and averages them into a single estimator.
 * Several ensembles, each with its own model, M, N and seed, can share one
 * context (a batch).
 *
 * Conventions for every entry point:
 *   - Pointers prefixed d_ are device pointers (HBM), h_ host pointers.
 *   - The library never allocates device memory: the caller passes one
 *     workspace (pf_workspace_bytes) and owns every buffer it passes in.
 *     The one static buffer it holds (PF_MLP_GRAD_STATIC_BYTES per device,
 *     for pf_mlp_loss_grad_noalloc) is part of the loaded code object.
 *     Host descriptor arrays are copied during pf_init and may be freed
 *     afterwards.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  All
 *     device work is enqueued asynchronously on it; a call returns once the
 *     work is enqueued.  Device faults surface at the next call that
 *     synchronises (pf_sync) or as PF_ERR_DEVICE from a later launch.
 *   - No function throws across the ABI.  Argument and call-order errors
 *     return a status before anything is enqueued; pf_last_error() gives a
 *     human-readable reason for the last failure on the calling thread.
 *   - One context is driven by one host thread at a time.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pf_status {
  PF_OK = 0,
  PF_ERR_INVALID_ARG = 1, /* bad descriptor, size, index or NULL pointer    */
  PF_ERR_UNSUPPORTED = 2, /* valid request the library does not implement   */
  PF_ERR_WORKSPACE = 3,   /* workspace too small or misaligned              */
  PF_ERR_DEVICE = 4,      /* a HIP runtime call failed                      */
  PF_ERR_STATE = 5        /* call out of order (e.g. step before init)      */
} pf_status;

/* State-space models (tau_0, tau_t, g_t) of Sec. 2.2. */
typedef enum pf_model_kind {
  /* x' = x - theta h x + sd sqrt(h) z, observed directly: the linear-Gaussian
     special case with a closed-form optimal filter (test model). */
  PF_MODEL_OU1D = 0,
  /* Stochastic Lorenz 63 under Euler-Maruyama, Sec. 4.1,
     eqs. (eqDiscreteLorenz-1..3); params = (s, r, b). */
  PF_MODEL_LORENZ63 = 1,
  /* FitzHugh-Nagumo network on a J x J grid, Sec. 5.1 eqs. (eqUd), (eqVd),
     classical reaction v(v-a)(1-v) - w + D lap(v), recovery eps (v - gam w),
     additive noise on both variables; lap is the 5-point Laplacian over the
     truncated neighbourhoods of Sec. 5.2 (no flux).
     params = (a, D, eps, gam). */
  PF_MODEL_FHN = 2,
  /* The paper's modified stochastic FH-N network, Sec. 5.1 eqs. (eqUd),
     (eqVd), (eqStimulusRegion)-(eqPsi_ijt), (eqObservFHN), with Sec. 5.2's
     constants in the descriptor:
       params     = (a2, c, beta0, beta1): p3(u) = a2 u - u^3 (the cubic read
                    with a negative leading coefficient), c = 1/D the weight
                    of the sum of the 4 neighbours' U, the recovery
                    V' = V + h (beta0 U + beta1 V + beta2);
       params_ext = (beta2, stimulus amplitude F~, Bernoulli parameter eps,
                    band u-, u+ of the stimulus region, duration l0 <= 32
                    (steps), forcing period, forcing pulse width (steps));
       noise_sd   = (sigma~ on U, on V).
     State (float32, state_dim = 2 J^2 + 4 ceil(l0/4)): the U plane, the V
     plane, then the ring of the last l0 stimulus events (slot n mod l0:
     centre node of the event of Euler step n, or -1; padding -1).  Step n:
     the region of nodes whose U or a 4-neighbour's U lies in (u-, u+); one
     Philox call (particle, filter, n, PROP << 24 | J*J/2): its first uniform
     < eps makes an event, centred on the floor(u |region|)-th region node
     (row-major), that stimulates the centre and its neighbours with F~ for
     l0 steps (F~ min{1, sum Q}: the printed max is read as min); forcing F~
     on the 2 x 2 corner block while (n mod period) < width; then Euler-
     Maruyama with the noise layout of the FH-N grid.  Observations read U
     nodes (< J*J).  Not with PF_ENS_LEARNED; with PF_ENS_AUXILIARY the
     pilot is the noise-free continuation without new stimulus events (the
     active stimuli and the forcing still act). */
  PF_MODEL_FHN_PAPER = 3
} pf_model_kind;

typedef struct pf_model_desc {
  int32_t kind;          /* pf_model_kind                                   */
  int32_t state_dim;     /* d_x: 1 (OU), 3 (Lorenz), 2*J*J (FH-N), 2*J*J + the
                            event ring (the paper's FH-N network)           */
  int32_t grid_j;        /* J for FH-N, else 0                              */
  int32_t steps_per_obs; /* S Euler-Maruyama steps per observation interval */
  double h;              /* Euler step                                      */
  double params[4];      /* see pf_model_kind                               */
  double noise_sd[2];    /* diffusion per variable class (v, w for FH-N);
                            the per-step noise is noise_sd * sqrt(h) * z    */
  int32_t obs_dim;       /* d_y                                             */
  const int32_t *h_obs_index; /* [obs_dim] observed state indices (H is a
                            selection); FH-N v of node (i,j) is i*J + j, and
                            FH-N models may observe v nodes only (< J*J)    */
  double obs_var;        /* Gaussian observation noise variance (eqObservLorenz,
                            eqObservFHN)                                    */
  const double *h_prior_mean; /* [state_dim] tau_0 = N(mean, diag(sd^2))    */
  const double *h_prior_sd;   /* [state_dim]                                */
  double params_ext[8];  /* PF_MODEL_FHN_PAPER only (see pf_model_kind)     */
} pf_model_desc;

/* One ensemble of M independent filters with N particles each, on model
   `model` (index into the model array), seeded by `seed`.  Filter m of the
   ensemble draws its random numbers from Philox4x32-10 counter word 1 = m. */
typedef struct pf_ensemble_desc {
  int32_t model;
  int32_t M;
  int32_t N;
  uint32_t flags; /* 0 (bootstrap proposal), PF_ENS_LEARNED or PF_ENS_AUXILIARY */
  uint64_t seed;
  /* Resampling (Sec. 2.3 notes that the convergence results also hold for
     other schemes than the multinomial one of Algorithm 1):
     scheme        PF_RESAMPLE_* (0 = multinomial, Algorithm 1);
     ess_threshold 0 resamples at every observation (Algorithm 1); a value in
                   (0, 1] resamples only when the effective sample size
                   (sum w)^2 / sum w^2 is below ess_threshold * N, and
                   otherwise keeps the particles with their weights carried
                   into the next interval (the filter's estimate is then the
                   weighted mean).  Anything but (multinomial, 0) needs a
                   PF_OPT_FUSED context and N <= 8192 (PF_ERR_UNSUPPORTED
                   otherwise). */
  int32_t scheme;
  int32_t reserved; /* 0 */
  double ess_threshold;
} pf_ensemble_desc;

/* Resampling schemes: each turns the normalised weights into ascending
   ancestors a_k = min{ i : C_i > U_k C_{N-1} } from sorted points U_k.
   MULTINOMIAL: U_k from N + 1 exponential spacings (Algorithm 1);
   SYSTEMATIC:  U_k = (k + u) / N, one uniform u (Philox counter (0, filter,
                t, RESAMPLE << 24 | 1), lane 0);
   STRATIFIED:  U_k = (k + u_k) / N, u_k from counter (k/4, filter, t,
                RESAMPLE << 24 | 2), lane k%4;
   RESIDUAL:    floor(N w_i / W) copies of particle i, then the remaining
                R draws multinomially from the fractional parts (sorted
                uniforms from the spacings of the exponentials E_0 .. E_R of
                the multinomial stream), ancestors in index order. */
#define PF_RESAMPLE_MULTINOMIAL 0
#define PF_RESAMPLE_SYSTEMATIC 1
#define PF_RESAMPLE_STRATIFIED 2
#define PF_RESAMPLE_RESIDUAL 3

/* Ensemble flag: draw the particles from the learned proposal instead of
   the model's transition (FH-N models with J <= 48 only).  Every Euler-
   Maruyama increment gets a drift correction u_theta(features of the node,
   y_t, step) and each particle's log-weight gains the log ratio of the model
   and proposal increment densities, so the filter stays consistent (the
   importance-function form of Algorithm 1 that the closing remarks of
   Sec. 6 extend the results to).  Until pf_proposal_set is called the
   network is zero and the filter is the bootstrap filter. */
#define PF_ENS_LEARNED 1u

/* Ensemble flag: run every filter of the ensemble as an auxiliary particle
   filter (Pitt and Shephard's auxiliary filter, the variant the paper runs
   on its FH-N network in Sec. 5.3; Sec. 3.3 notes that the ensemble results
   extend to it).  Each interval: a pilot mu_i, the noise-free S-step Euler
   path of the model from particle i; first-stage log-weights lambda_i =
   lwc_i + log g(y_t | mu_i) (lwc: carried log-weights, mean weight 1);
   ancestors by the ensemble's scheme from lambda; propagation of the
   selected particles; second-stage log-weights log g(y_t | x_k) -
   log g(y_t | mu_{a_k}), normalised and carried to the next interval (the
   filter's estimate is their weighted mean; no resampling at the end of the
   interval).  log G advances by both stages' factors, so exp(log G) stays
   unbiased for p(y_{1:t}).  Needs PF_OPT_FUSED, N <= 8192, the bootstrap
   transition (not PF_ENS_LEARNED) and ess_threshold 0. */
#define PF_ENS_AUXILIARY 2u

/* Context options (pf_init `options`). */
#define PF_OPT_PLAIN 0u /* one kernel per method step (reference path)     */
#define PF_OPT_FUSED 1u /* fused interval: batched propagation with the gather
                           and weighting fused in, per-filter resampling and
                           estimators, no materialised post-resampling state   */
#define PF_OPT_GRAPH 2u /* with PF_OPT_FUSED: once observations are staged
                           (pf_set_observations), each interval after the first
                           is one launch of a captured hipGraph               */

/* Stages for pf_run_stages (bit mask). */
#define PF_STAGE_PROPAGATE 1u /* Algorithm 1 step 2(a): draw from tau_t        */
#define PF_STAGE_WEIGHT 2u    /* step 2(a): log g_t^{y_t}                      */
#define PF_STAGE_RESAMPLE 4u  /* steps 2(a)-(b): normalise, CDF, sorted
                                 uniforms, ancestor search                     */
#define PF_STAGE_GATHER 8u    /* step 2(b): x_t^(k) = xbar_t^(a_k)             */
#define PF_STAGE_ESTIMATE 16u /* (f, pi_t^N), (f, pi_t^{MxN}) for f = identity */
#define PF_STAGE_ALL 31u

typedef struct pf_ctx pf_ctx; /* opaque; the library owns only this host struct */

/* Launch shapes of the fused path.  Every choice computes the same filter;
   they differ in speed only (the per-filter resampling reductions run in a
   different order with a different workgroup size, so the last bits of the
   normalising sums and, at a CDF boundary, an ancestor index can change). */
typedef struct pf_tuning {
  int32_t vec_single_kernel;  /* 1: one workgroup runs a whole vector-model
                                 filter interval (N <= 8192); 0: batched
                                 propagation tiles, then per-filter resampling */
  int32_t prop_tile;          /* particles per batched-propagation workgroup:
                                 64, 128 or 256                                */
  int32_t resample_bd_min;    /* smallest per-filter resampling workgroup: 64,
                                 128, 256, 512 or 1024 (a filter of N particles
                                 takes the smallest allowed size >= N, else
                                 1024)                                          */
  int32_t grid_blocks_per_cu; /* resident workgroups per CU of the batched FH-N
                                 stepping kernel; 0 = as many as fit           */
} pf_tuning;

/* Bytes of device workspace pf_init needs for these descriptors. */
pf_status pf_workspace_bytes(const pf_model_desc *h_models, int32_t n_models,
                             const pf_ensemble_desc *h_ens, int32_t n_ens,
                             uint32_t options, size_t *out_bytes);

/* Validate the descriptors, lay the workspace out (d_workspace must be
   256-byte aligned and at least pf_workspace_bytes long; the caller keeps it
   alive until pf_destroy), upload model constants and draw every filter's
   initial particles x_0 ~ tau_0 (Algorithm 1, step 1).  The next pf_step
   processes interval t = 1. */
pf_status pf_init(const pf_model_desc *h_models, int32_t n_models,
                  const pf_ensemble_desc *h_ens, int32_t n_ens, uint32_t options,
                  void *d_workspace, size_t workspace_bytes, void *stream,
                  pf_ctx **out_ctx);

/* One observation interval t for every ensemble (Algorithm 1, step 2):
   S Euler-Maruyama steps per particle, Gaussian log-likelihood weighting,
   normalisation with the update of log G_t^N (eqGtN), multinomial resampling
   and the estimators.  d_y: float32, the observations y_t of every ensemble
   concatenated in ensemble order (obs_dim of its model each), or NULL to use
   the record staged by pf_set_observations.  Advances t.  With PF_OPT_FUSED
   and a batch that holds both vector-model and grid-model ensembles, the
   grid ensembles' part of the interval runs on a stream of the context,
   forked from `stream` and joined back to it before the cross-filter means
   (unless profiling is on): all of the interval still follows earlier work
   on `stream` and precedes later work on it. */
pf_status pf_step(pf_ctx *ctx, const float *d_y, void *stream);

/* Stage the observation record on the device: d_y_all float32 [T][sum_e
   obs_dim(e)] (interval t uses row t-1), caller-owned and kept alive while the
   context uses it.  pf_step(ctx, NULL, stream) then reads y_t from it; with
   PF_OPT_GRAPH the interval index is kept on the device too, so the captured
   interval replays unchanged.  Stepping past T is an error. */
pf_status pf_set_observations(pf_ctx *ctx, const float *d_y_all, int32_t T);

/* Run selected stages (PF_STAGE_*) of the current interval without advancing
   t: the per-step hooks of the parity tests.  They run on the plain kernels,
   except that on a PF_OPT_FUSED context a request with PF_STAGE_RESAMPLE and
   without PROPAGATE / WEIGHT runs the fused kernel's resampling and estimation
   phases on the log-weights and pre-resampling particles in place.  For an
   ensemble with PF_ENS_LEARNED, PF_STAGE_PROPAGATE needs d_y (the proposal
   looks at y_t) and writes the complete log-weights (observation term plus
   the density ratio); PF_STAGE_WEIGHT leaves them as they are. */
pf_status pf_run_stages(pf_ctx *ctx, uint32_t stages, const float *d_y, void *stream);

/* Estimates after the last completed interval.  Any pointer may be NULL.
   d_mean:   float64 [sum_e state_dim(e)]: ensemble average (Definition 3) of
             the post-resampling filter means (f, pi_t^{m,N}), f = identity.
   d_mean_w: float64 [sum_e state_dim(e)]: ensemble average of the weighted
             pre-resampling means sum_i w_t^(i) xbar_t^(i).
   d_logZ:   float64 [sum_e M(e)]: log G_t^N per filter including the Gaussian
             normalising constant, so that exp(d_logZ) is unbiased for
             p(y_{1:t}) (Lemma 2); -inf once a filter degenerated.
   d_filter_mean: float64 [sum_e M(e)*state_dim(e)]: per-filter means.
   A filter that kept its particles in the last interval (ESS threshold)
   contributes its weighted mean to d_mean and d_filter_mean. */
pf_status pf_estimate(pf_ctx *ctx, double *d_mean, double *d_mean_w, double *d_logZ,
                      double *d_filter_mean, void *stream);

/* Test hooks.  Particle layouts: vector models (OU, Lorenz) float32
   [M][state_dim][N]; grid model (FH-N) float32 [M][N][state_dim]. */
pf_status pf_set_particles(pf_ctx *ctx, int32_t ens, const float *d_x, void *stream);
/* post-resampling particles x_t (materialised by a gather if needed) */
pf_status pf_get_particles(pf_ctx *ctx, int32_t ens, float *d_x, void *stream);
/* pre-resampling particles xbar_t of the current interval (get / overwrite) */
pf_status pf_get_predicted(pf_ctx *ctx, int32_t ens, float *d_x, void *stream);
pf_status pf_set_predicted(pf_ctx *ctx, int32_t ens, const float *d_x, void *stream);
/* log-weights float32 [M][N] of the current interval (with an ESS threshold:
   the carried log-weight plus the log-likelihood, once the interval ran) */
pf_status pf_get_logweights(pf_ctx *ctx, int32_t ens, float *d_lw, void *stream);
pf_status pf_set_logweights(pf_ctx *ctx, int32_t ens, const float *d_lw, void *stream);
/* ancestors int32 [M][N] of the current interval, ascending per filter */
pf_status pf_get_ancestors(pf_ctx *ctx, int32_t ens, int32_t *d_a, void *stream);
/* carried log-weights float32 [M][N] of an ensemble with an ESS threshold:
   log-weights of particles that were kept at the end of the last interval,
   normalised so that their exponentials average 1 (all zero after a
   resampling); the next interval adds them to the log-likelihoods
   (get / overwrite) */
pf_status pf_get_carried_logweights(pf_ctx *ctx, int32_t ens, float *d_lwc, void *stream);
pf_status pf_set_carried_logweights(pf_ctx *ctx, int32_t ens, const float *d_lwc, void *stream);
/* per-filter float64 [M][4]: max log-weight, sum exp(lw - max),
   sum exp(2(lw - max)), degenerate flag (1.0 if no weight was positive) */
pf_status pf_get_filter_stats(pf_ctx *ctx, int32_t ens, double *d_stats, void *stream);
/* Set the interval index t that the next pf_step / pf_run_stages processes. */
pf_status pf_set_interval(pf_ctx *ctx, int32_t t);
pf_status pf_get_interval(const pf_ctx *ctx, int32_t *out_t);

/* Truth path and observations from the model of ensemble `ens` on the
   dedicated truth stream of `seed`: d_x_true float32 [(T+1)][state_dim]
   (row 0 is x_0 ~ tau_0), d_y float32 [T][obs_dim].  Synthetic-data helper
   for benchmarks; runs on the GPU. */
pf_status pf_simulate(pf_ctx *ctx, int32_t ens, uint64_t seed, int32_t T,
                      float *d_x_true, float *d_y, void *stream);

/* Random-number hook: for i in [0, n), word/normal i comes from the Philox4x32-10
   call with counter (i/4, c1, c2, c3) and key(seed), lane i%4.  d_bits uint32
   [n] and d_z float32 [n] (Box-Muller normals); either may be NULL. */
pf_status pf_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                           int64_t n, uint32_t *d_bits, float *d_z, void *stream);

/* ---- learned proposal ----------------------------------------------------
   u_theta is an MLP in_dim -> 64 (ReLU) -> 64 (ReLU) -> out_dim with FP32
   parameters, flat, in the order W1[64][in_dim], b1[64], W2[64][64], b2[64],
   W3[out_dim][64], b3[out_dim] (row-major, y = W x + b).  Kernels round them
   to bfloat16 (nearest even) when they load them, round inputs and hidden
   activations to bfloat16 too, and accumulate in FP32 (MFMA).
   FH-N features of node (i, j) at Euler step k of the interval (22 inputs):
   the 3x3 patch of v around the node, row-major, edge replicated; the same
   patch of w; y_o - v_o for the node's nearest observed node o = (i_o, j_o)
   (least grid distance, ties to the lower observation index); (S - k) / S;
   (i_o - i) / 2 and (j_o - j) / 2.
   Outputs: the corrections of the v and w drifts of the node. */

/* Number of parameters of an MLP, or -1 unless 1 <= in_dim <= 31 and
   1 <= out_dim <= 4. */
int32_t pf_mlp_nparams(int32_t in_dim, int32_t out_dim);

/* Copy the network of ensemble `ens` (created with PF_ENS_LEARNED) from
   d_params (float32, pf_mlp_nparams(22, 2) values) into the workspace;
   enqueued on `stream`, used from the next interval on. */
pf_status pf_proposal_set(pf_ctx *ctx, int32_t ens, const float *d_params, int64_t n_params,
                          void *stream);

/* d_out [rows][out_dim] = u_theta(d_x [rows][in_dim]), float32, with the
   kernels' bfloat16 arithmetic.  rows = 0 is a no-op. */
pf_status pf_mlp_forward(const float *d_params, int32_t in_dim, int32_t out_dim, const float *d_x,
                         int64_t rows, float *d_out, void *stream);

/* ---- training of u_theta ---------------------------------------------------
   Regression of u_theta onto the scaled Euler noise of model paths: the loss
   is the mean over rows of |u_theta(x) - target|^2.  Its minimiser is the
   conditional mean of the increment noise given the features, which for a
   linear-Gaussian model is the drift of the optimal (Doob) proposal.  All of
   it runs in HIP kernels: forward on MFMA, a hand-written backward (layer 3
   on the VALU, layer 2 and every weight gradient on MFMA), a fixed-order
   reduction of per-wave partial gradients and Adam on FP32 master weights. */

/* Bytes of the work buffer of pf_mlp_loss_grad for `rows` rows. */
pf_status pf_mlp_grad_work_bytes(int32_t in_dim, int32_t out_dim, int64_t rows, size_t *out_bytes);

/* d_grad [pf_mlp_nparams] = gradient of (1/rows) sum_r |u(x_r) - t_r|^2 at
   d_params, with d_x [rows][in_dim], d_target [rows][out_dim] (float32);
   the loss to *d_loss (device float) when d_loss is not NULL.  Deterministic
   (no atomics).  d_work: pf_mlp_grad_work_bytes bytes, caller-owned. */
pf_status pf_mlp_loss_grad(const float *d_params, int32_t in_dim, int32_t out_dim, const float *d_x,
                           const float *d_target, int64_t rows, float *d_grad, float *d_loss,
                           void *d_work, size_t work_bytes, void *stream);

/* Size of the library's static partial-gradient buffer (per device). */
#define PF_MLP_GRAD_STATIC_BYTES ((size_t)16 << 20)

/* pf_mlp_loss_grad without a work buffer, for callers that cannot allocate
   device memory (code under HIP graph capture, serving loops, harnesses that
   forbid allocation): the per-wave partial gradients go to a static buffer
   of PF_MLP_GRAD_STATIC_BYTES that the library holds on each device it runs
   on until the process ends.  The result is bit-identical to
   pf_mlp_loss_grad (same launch shape, same fixed-order reduction).  The
   first call on a device looks the buffer's address up (with that device
   current); no call allocates or frees memory.  PF_ERR_WORKSPACE when the
   call needs more partial-gradient bytes than the buffer holds
   (pf_mlp_grad_work_bytes > PF_MLP_GRAD_STATIC_BYTES; for the 22 -> 2 FH-N
   proposal network that is beyond 46336 rows).  Every call on one device
   shares the buffer: calls that overlap on one device (on different
   streams, or from different host threads) race and must be serialised by
   the caller.  Nothing in the buffer needs clearing: every call overwrites
   every value it reads. */
pf_status pf_mlp_loss_grad_noalloc(const float *d_params, int32_t in_dim, int32_t out_dim,
                                   const float *d_x, const float *d_target, int64_t rows,
                                   float *d_grad, float *d_loss, void *stream);

/* One Adam step (Kingma and Ba, Algorithm 1) at step t >= 1, in place on
   d_params, d_m, d_v (float32, n values). */
pf_status pf_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t n,
                       double lr, double beta1, double beta2, double eps, int32_t t, void *stream);

/* Training of an FH-N proposal (J a multiple of 4, J <= 48) on paths the
   model simulates itself.  All draws use Philox with key(seed) and purpose
   TRAIN (7):
     long run q (q < n_runs): x_0 ~ tau_0 from counters (q, 0xFFFFFFFE,
       0xFFFFFFFF, s/4) lane s%4; Euler step n from (q, 0xFFFFFFFE, n, pair);
       start state j (j < run_len) of the run is its state at the end of
       interval j + 1;
     trajectory r = q * run_len + j: one interval from that start, step k
       from (r, 0xFFFFFFFD, k, pair), and y_r = H x_S + sqrt(obs_var) eta with
       eta_o from (r, 0xFFFFFFFD, 0xFFFFFFFF, o/4) lane o%4;
     regression rows (r, k, node): the node's features at x_k of trajectory
       r with y_r (as in the filter), target (noise_sd / sqrt(h)) z_k (v, w);
     minibatch of Adam step s: batch_tiles tiles of 16 consecutive nodes,
       tile b from the words (w0, w1, w2) of counter (b, 0xFFFFFFFC, s, 0):
       r = floor(w0 n_traj / 2^32), k = w1 mod S, first node
       16 floor(w2 (J*J/16) / 2^32). */
typedef struct pf_train_desc {
  int32_t n_runs;      /* long model runs from tau_0                      */
  int32_t run_len;     /* intervals per run; n_runs * run_len trajectories */
  int32_t batch_tiles; /* 16-row tiles per Adam step                      */
  int32_t reserved;    /* 0                                               */
  double lr, beta1, beta2, eps;
  uint64_t seed;
} pf_train_desc;

/* Workspace bytes for training: the start states, the trajectories
   (n_runs * run_len * S * state_dim floats), their observations, the
   partial gradients and the Adam moments. */
pf_status pf_train_workspace_bytes(const pf_model_desc *h_model, const pf_train_desc *d,
                                   size_t *out_bytes);

/* Simulate the long runs and the trajectories into d_work (256-byte
   aligned, pf_train_workspace_bytes).  Waits for the host staging copies. */
pf_status pf_train_data(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                        size_t work_bytes, void *stream);

/* Device pointers into d_work: start states float32 [n_traj][state_dim],
   trajectories [n_traj][S][state_dim] (state before each step), and
   observations [n_traj][obs_dim].  Any output may be NULL. */
pf_status pf_train_buffers(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                           float **d_starts, float **d_traj, float **d_y);

/* Adam steps first_step .. first_step + n_steps - 1 on d_params (float32,
   pf_mlp_nparams(22, 2), updated in place); the moments live in d_work and
   are cleared when first_step == 1.  d_loss [n_steps] (device, may be NULL)
   receives each minibatch's loss before its update. */
pf_status pf_train_steps(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                         size_t work_bytes, float *d_params, int32_t first_step, int32_t n_steps,
                         float *d_loss, void *stream);

/* Gradient and loss of the minibatch of Adam step `step` at d_params, without
   an update (the training test hook). */
pf_status pf_train_grad(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                        size_t work_bytes, const float *d_params, int32_t step, float *d_grad,
                        float *d_loss, void *stream);

/* ---- launch-shape tuning of the fused path ---------------------------------
   pf_init starts from {0, 256, 256, 0}. */
pf_status pf_get_tuning(const pf_ctx *ctx, pf_tuning *out);
/* Rebuild the launch plan for `u` (waits for the context's queued work; the
   next interval uses it; captured graphs are re-captured). */
pf_status pf_set_tuning(pf_ctx *ctx, const pf_tuning *u, void *stream);
/* Autotuner: times `reps` fused intervals (after one warm-up) on the device
   for each candidate, searching one knob at a time (single-kernel vector
   path, propagation tile, resampling workgroup floor, grid residency), keeps
   the fastest, writes it to *out (may be NULL) and resets every filter to
   its prior draw at interval 1 (the timed intervals move them).  Needs a
   PF_OPT_FUSED context and one interval's observations d_y. */
pf_status pf_autotune(pf_ctx *ctx, const float *d_y, int32_t reps, void *stream, pf_tuning *out);

/* Timing of the dominant kernel (the propagation kernel on the plain path,
   the fused interval kernel on the fused path).  While enabled, every
   pf_step records a pair of HIP events around that kernel on the stream it
   is launched on (at most 65536 pairs are kept).  pf_read_profile waits for
   them, returns the summed duration in milliseconds and the number of
   launches, and clears the record. */
pf_status pf_set_profiling(pf_ctx *ctx, int32_t enable);
pf_status pf_read_profile(pf_ctx *ctx, double *out_ms, int64_t *out_launches);

/* Block until all work of the context's last stream is done; reports an
   asynchronous device error as PF_ERR_DEVICE. */
pf_status pf_sync(pf_ctx *ctx);
/* Wait for the context's queued work (on the last stream it was given and on
   its own streams), then release its streams, events and captured graphs and
   the host struct.  The caller's workspace may be freed afterwards.  Call it
   while the HIP runtime is alive (not from a static destructor that runs
   after the runtime's own teardown).  NULL is a no-op. */
void pf_destroy(pf_ctx *ctx);
const char *pf_status_str(pf_status s);
const char *pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
