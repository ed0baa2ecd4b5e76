/*
 * pf_oracle.h -- plain, slow, single-threaded FP64 reference of the
 * independent-ensemble bootstrap particle filter (Crisan, Miguez, Rios,
 * arXiv 1407.8071).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path: the Philox
 * generator, Box-Muller, the model drifts, the resampler and the estimators
 * are written here a second time, from their published definitions.
 *
 * What is computed, and where the paper defines it:
 *   - state-space model (tau_0, tau_t, g_t): Sec. 2.2, eqs. (eqPrior),
 *     (eqKernel) and the conditional observation density g_t;
 *   - bootstrap filter: Sec. 2.3, Algorithm 1 (initialise from tau_0; per
 *     observation draw from tau_t, weight by g_t and normalise, resample
 *     multinomially);
 *   - normalising-constant estimate G_t^N: Sec. 2.3, eq. (eqGtN);
 *   - estimators (f, xi_t^N), (f, pi_t^N): Sec. 2.3 (sample averages);
 *   - ensemble measure pi_t^{MxN} = (1/M) sum_m pi_t^{m,N}: Sec. 3.3,
 *     Definition 3;
 *   - stochastic Lorenz 63 under Euler-Maruyama: Sec. 4.1,
 *     eqs. (eqDiscreteLorenz-1..3) and (eqObservLorenz);
 *   - FitzHugh-Nagumo grid: Sec. 5.1, eqs. (eqUd), (eqVd) with the
 *     neighbourhoods of Sec. 5.2 (classical reaction term, see DESIGN
 *     readings), observations eq. (eqObservFHN);
 *   - 1-D Ornstein-Uhlenbeck test model and its exact Kalman filter: the
 *     linear-Gaussian special case of Sec. 2.2 in which the recursion
 *     (eqRecursiveFormula1) has a closed form.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed and countered as described in
 * the comments of pf_oracle.c; uniforms u = (2*(x>>9)+1) * 2^-24 in (0,1);
 * normals by the Box-Muller transform; exponential variates -ln u.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OU1D = 0, OR_LORENZ63 = 1, OR_FHN = 2, OR_FHN_PAPER = 3 };

/* Counter "purpose" tags (top byte of counter word 3). */
enum {
  OR_P_INIT = 1, OR_P_PROP = 2, OR_P_RESAMPLE = 3, OR_P_TRUTH_INIT = 4,
  OR_P_TRUTH_NOISE = 5, OR_P_OBS_NOISE = 6, OR_P_TRAIN = 7, OR_P_CONFIG = 8
};

#define OR_TRUTH_STREAM 0xFFFFFFFFu

typedef struct {
  int kind;                 /* OR_OU1D, OR_LORENZ63, OR_FHN                    */
  int dx;                   /* state dimension (FHN: 2*J*J, v plane then w)    */
  int J;                    /* grid side (FHN only)                            */
  int S;                    /* Euler-Maruyama steps per observation interval  */
  double h;                 /* Euler step                                      */
  double p[4];              /* OU: theta | L63: s, r, b | FHN: a, D, eps, gam  */
  double sd[2];             /* diffusion coefficient per variable class        */
  int dy;                   /* observation dimension                           */
  const int *obs_idx;       /* [dy] observed state indices (H is a selection)  */
  double obs_var;           /* observation noise variance                      */
  const double *prior_mean; /* [dx]                                            */
  const double *prior_sd;   /* [dx]                                            */
  double q[8];              /* OR_FHN_PAPER: beta2, stimulus amplitude F~,
                               Bernoulli parameter eps, thresholds u-, u+,
                               stimulus duration l0 (steps), forcing period and
                               pulse width (steps)                             */
} or_model;

/* ---- the paper's modified FH-N network (Sec. 5.1, 5.2) -----------------
   State of a particle: the U plane [J*J], the V plane [J*J], then a ring of
   the last l0 stimulus events (slot n mod l0 holds the event of step n: the
   centre node i*J+j of the stimulated group, or -1), padded with -1 to a
   multiple of 4 (dx = 2 J^2 + 4 ceil(l0/4)).  p = (a2, c, beta0, beta1) with
   p3(u) = a2 u - u^3 (read with a negative leading coefficient: the printed
   sign gives no rest state), c = 1/D the coupling of the neighbour sum
   (eqUd), (beta0, beta1, beta2) the recovery (eqVd); sd = (sigma~, 0).
   Step n (0-based; the paper's t = n + 1) from U, V:
     1. the stimulus region S (eqStimulusRegion): nodes with U in (u-, u+)
        at the node or one of its 4 grid neighbours;
     2. one Philox call (c0, c1, n, purpose | sub-block J*J/2): u0 < eps is
        the Bernoulli event (eqBernu), u1 picks the centre uniformly from S
        in row-major order, floor(u1 |S|) (eqUnifStimulus); no event when S
        is empty;
     3. the event enters the ring, replacing the event of step n - l0;
     4. Psi = F~ on every node covered by an event of the ring (the centre or
        one of its 4 neighbours), else 0 -- F~ min{1, sum_l Q} (eqPsi_ijt,
        whose max is read as min: the printed max keeps every node
        stimulated);
     5. forcing m F_n: F~ on the 2 x 2 corner block (i, j < 2) while
        (n mod period) < width, else 0 (the printed square pulse spans the
        whole period);
     6. Euler (eqUd, eqVd): U' = U + h (p3(U) - V) + h (c sum_nbr U + m F +
        Psi) + sigma~ sqrt(h) z, V' = V + h (beta0 U + beta1 V + beta2). */
int or_fhnp_region(const or_model *m, const double *U, int *region);
/* one step of the network (x, xo of dx); returns the event centre or -1 */
int or_fhnp_step(const or_model *m, const uint32_t key[2], uint32_t purpose, uint32_t c0,
                 uint32_t c1, uint32_t n, const double *x, double *xo);
/* the noise-free continuation of step n (the auxiliary filter's pilot):
   the Euler step with z = 0; for the FH-N network also no new stimulus
   event (active stimuli and the forcing still act) */
void or_pilot_step(const or_model *m, uint32_t n, const double *x, double *xo);
/* one step of any model: normals and the Euler-Maruyama step, and the
   stimulus process of the paper's network */
void or_transition(const or_model *m, const uint32_t key[2], uint32_t purpose, uint32_t c0,
                   uint32_t c1, uint32_t n, const double *x, double *xo);

/* ---- random numbers ---------------------------------------------------- */
void or_key(uint64_t seed, uint32_t key[2]);
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u01(uint32_t x);
void or_normals4(const uint32_t ctr[4], const uint32_t key[2], double z[4]);
/* bulk helpers for statistical tests: n words / normals from counters
   (c0 = i/4 for i in [0,n), c1, c2, c3 fixed), lane i%4. */
void or_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, uint32_t *out);
void or_normal_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, double *out);

/* ---- model ------------------------------------------------------------- */
void or_drift(const or_model *m, const double *x, double *f);
void or_laplacian(int J, const double *v, double *lap);
/* normals of Euler step n for (c0, c1) under `purpose`: z[dx] */
void or_step_noise(const or_model *m, const uint32_t key[2], uint32_t purpose,
                   uint32_t c0, uint32_t c1, uint32_t n, double *z);
void or_em_step(const or_model *m, const double *x, const double *z, double *xo);
void or_prior_draw(const or_model *m, const uint32_t key[2], uint32_t purpose,
                   uint32_t c0, uint32_t c1, double *x);
double or_loglik(const or_model *m, const double *x, const double *y);

/* ---- filter steps (one filter, N particles, X is [N][dx]) -------------- */
void or_init(const or_model *m, uint64_t seed, uint32_t filter, int N, double *X);
void or_propagate(const or_model *m, uint64_t seed, uint32_t filter, int N,
                  int t, double *X);
void or_propagate_particle(const or_model *m, uint64_t seed, uint32_t filter,
                           uint32_t index, int t, double *x);
void or_weights(const or_model *m, int N, const double *X, const double *y,
                double *lw);
/* returns mx, W = sum exp(lw-mx), sumw2 = sum exp(2(lw-mx)); degenerate flag */
int or_normalise(int N, const double *lw, double *mx, double *W, double *sumw2);
/* effective sample size (sum w)^2 / sum w^2 of the weights exp(lw) */
double or_ess(int N, const double *lw);
void or_cdf(int N, const double *lw, double mx, int degenerate, double *C);
void or_sorted_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U);
void or_ancestors(int N, const double *C, const double *U, int32_t *A);
void or_gather(int N, int dx, const double *X, const int32_t *A, double *Xo);
void or_mean(int N, int dx, const double *X, double *mean);
void or_weighted_mean(int N, int dx, const double *X, const double *lw,
                      double mx, double *mean);

/* One observation interval of one filter: propagate, weight, normalise,
   resample, estimate.  X [N][dx] is updated in place (post-resampling).
   Outputs (any may be NULL): lw[N], A[N], mean_post[dx], mean_w[dx].
   logZ is incremented by log of the interval's factor of G_t^N including the
   Gaussian normalising constant.  Returns 1 if the weights were degenerate. */
int or_filter_interval(const or_model *m, uint64_t seed, uint32_t filter, int N,
                       int t, double *X, const double *y, double *logZ,
                       double *lw, int32_t *A, double *mean_post,
                       double *mean_w, double *ess);

/* ---- other resampling schemes and the ESS-triggered schedule ------------
   Sec. 2.3 notes that the convergence results also hold for other resampling
   schemes than multinomial.  Each scheme turns the normalised weights into
   ascending ancestors a_k = min{ i : C_i > U_k C_{N-1} } from sorted points
   U_k in [0, 1):
     systematic: U_k = (k + u) / N with one uniform u (counter (0, filter, t,
                 RESAMPLE | sub-block 1), lane 0);
     stratified: U_k = (k + u_k) / N with u_k from counter (k/4, filter, t,
                 RESAMPLE | sub-block 2), lane k%4;
     residual:   n_i = floor(N w_i / W) copies of particle i, then R = N -
                 sum n_i multinomial draws from the residual weights
                 N w_i / W - n_i (sorted uniforms from the exponentials
                 E_0 .. E_R of the multinomial stream); the ancestors list
                 particle i its total number of times, in index order. */
enum { OR_RS_MULTINOMIAL = 0, OR_RS_SYSTEMATIC = 1, OR_RS_STRATIFIED = 2, OR_RS_RESIDUAL = 3 };
void or_systematic_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U);
void or_stratified_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U);
void or_residual_ancestors(uint64_t seed, uint32_t filter, int t, int N, const double *lw,
                           double mx, int degenerate, int32_t *A);
/* ancestors A[N] of the log-weights lw[N] by `scheme` */
void or_resample_scheme(int scheme, uint64_t seed, uint32_t filter, int t, int N,
                        const double *lw, int32_t *A);

/* One interval with a resampling scheme and schedule.  lwc[N] (in/out)
   holds the carried log-weights of the particles, normalised so that
   sum_i exp(lwc_i) = N (all zero after a resampling).  The particles'
   log-weights are lw_i = lwc_i + log g(y | xbar_i); log G advances by
   mx + log(W/N) + the Gaussian constant, as in or_filter_interval.  The
   filter resamples (by `scheme`) when ess_threshold <= 0 (every interval,
   Algorithm 1), when the weights are degenerate, or when the ESS
   (sum w)^2 / sum w^2 is below ess_threshold * N; then lwc = 0 and
   mean_est is the post-resampling mean.  Otherwise the particles stay
   (A = identity), lwc_i = lw_i - mx - log(W/N) and mean_est is the weighted
   mean.  *resampled receives the decision.  Outputs may be NULL. */
int or_filter_interval_sched(const or_model *m, uint64_t seed, uint32_t filter, int N, int t,
                             double *X, double *lwc, const double *y, double *logZ, int scheme,
                             double ess_threshold, double *lw, int32_t *A, double *mean_est,
                             double *mean_w, double *ess, int *resampled);

/* Auxiliary particle filter interval (Pitt and Shephard's auxiliary filter,
   the variant the paper runs on its FH-N network in Sec. 5.3; Sec. 3.3 notes
   that the ensemble results extend to it).  From the particles X[N] with
   carried log-weights lwc[N] (mean weight 1):
     1. pilot: mu_i = the noise-free S-step Euler path of the model from x_i
        (or_pilot_step);
        first-stage log-weights lambda_i = lwc_i + log g(y | mu_i);
     2. ancestors a_k by `scheme` from lambda (counters of interval t);
     3. propagation of x_{a_k} (the bootstrap's noise counters, slot k);
     4. second-stage log-weights lw_k = log g(y | x_k) - log g(y | mu_{a_k}),
        never resampled: lwc_k = lw_k - mx - log(W/N), and the estimate
        mean_w is the weighted mean sum_k w_k x_k / W.
   log G advances by the two stages' mx + log(W/N) and the Gaussian
   constant, so that exp(log G) stays unbiased for p(y_{1:t}).  Outputs may
   be NULL; A receives the first-stage ancestors.  Returns 1 if either
   stage's weights were degenerate. */
int or_apf_interval(const or_model *m, uint64_t seed, uint32_t filter, int N, int t, double *X,
                    double *lwc, const double *y, double *logZ, int scheme, double *lw,
                    int32_t *A, double *mean_w, double *ess);

/* Whole ensemble run over T observations y[T][dy].  est[T][dx] receives the
   ensemble (equal-weight) post-resampling mean, est_w[T][dx] the ensemble of
   weighted pre-resampling means, logZ[M] the final log-evidence per filter,
   ess[T] the mean ESS over filters.  Filter m uses Philox counter word 1 = m
   and the given seed.  Any output may be NULL. */
void or_run_ensemble(const or_model *m, uint64_t seed, int M, int N, int T,
                     const double *y, double *est, double *est_w,
                     double *logZ, double *ess);

/* Truth trajectory x_true[(T+1)][dx] (row 0 = x_0) and observations
   y[T][dy], from the truth stream of `seed`. */
void or_simulate(const or_model *m, uint64_t seed, int T, double *x_true,
                 double *y);

/* Exact Kalman filter for the OU test model observed every S steps:
   mean[T], var[T] of the filtering distributions and the log marginal
   likelihood log p(y_{1:T}). */
double or_kalman_ou(const or_model *m, int T, const double *y, double *mean,
                    double *var);

/* ---- learned proposal --------------------------------------------------
   A drift correction u_theta(features) added to every Euler increment:
   x' = x + h (f(x) + u) + sd sqrt(h) z, and the importance weight of the
   particle is multiplied by the ratio of the model and proposal Gaussian
   increment densities, log p/q = -(sqrt(h)/sd) u z - (h/(2 sd^2)) u^2 per
   component and step.  u_theta is an MLP in_dim -> 64 (ReLU) -> 64 (ReLU)
   -> out_dim (linear) with parameters, in this order, W1[64][in_dim],
   b1[64], W2[64][64], b2[64], W3[out_dim][64], b3[out_dim].
   FH-N features of node (i, j) at step k of the interval (22): the 3x3 v
   patch and the 3x3 w patch around the node (row-major offsets -1..1, edge
   replicated), the residual y_o - v_o of the nearest observed node o
   = (i_o, j_o), tau = (S - k) / S, and the offsets (i_o - i)/2, (j_o - j)/2;
   outputs (u_v, u_w).
   OU features (3): x, y - x, tau; output u. */
#define OR_MLP_HIDDEN 64
int or_mlp_nparams(int in_dim, int out_dim);
/* h1, h2 may be NULL.  bf16 != 0 rounds inputs, weights and hidden
   activations to bfloat16 (nearest even) before each layer. */
void or_mlp_forward(int in_dim, int out_dim, const double *p, const double *x,
                    double *h1, double *h2, double *out, int bf16);
/* grad += d(dout . out)/dp at input x (FP64, no rounding) */
void or_mlp_backward(int in_dim, int out_dim, const double *p, const double *x,
                     const double *dout, double *grad);
/* mean over B rows of sum_c (out_c - target_c)^2, and its gradient */
double or_mlp_loss_grad(int in_dim, int out_dim, const double *p, int B,
                        const double *X, const double *T, double *grad);
double or_bf16(double x);
/* nearest observed node of every node (ties to the lowest observation
   index), as an index into obs_idx */
void or_nearest_obs(const or_model *m, int *map);
void or_fhn_features(const or_model *m, const double *x, const double *y,
                     const int *nearest, int k, int node, double *feat);
void or_ou_features(const or_model *m, const double *x, const double *y, int k,
                    double *feat);
/* Interval t of N particles under the learned proposal (Philox counters of
   the bootstrap propagation, so p = 0 reproduces it); dlw[N] receives the
   log increment-density ratios. */
void or_propagate_learned(const or_model *m, const double *p, uint64_t seed,
                          uint32_t filter, int N, int t, double *X,
                          const double *y, double *dlw, int bf16);
/* The same draw for one particle (Philox counter word 0 = index), in place on
   x[dx]; returns its log increment-density ratio. */
double or_propagate_learned_particle(const or_model *m, const double *p, uint64_t seed,
                                     uint32_t filter, uint32_t index, int t, double *x,
                                     const double *y, int bf16);
/* One full interval of one filter under the learned proposal (as
   or_filter_interval). */
int or_filter_interval_learned(const or_model *m, const double *p, uint64_t seed,
                               uint32_t filter, int N, int t, double *X,
                               const double *y, double *logZ, double *lw,
                               int32_t *A, double *mean_post, double *mean_w,
                               double *ess, int bf16);
void or_run_ensemble_learned(const or_model *m, const double *p, uint64_t seed,
                             int M, int N, int T, const double *y, double *est,
                             double *est_w, double *logZ, double *ess, int bf16);
/* OU: the minimiser of E|u - (sd/sqrt(h)) z_k|^2 given x_k = x and y,
   sd^2 a_{S-k-1} (y - a_{S-k} x) / (q_{S-k} + obs_var), k 0-based. */
double or_ou_optimal_u(const or_model *m, double x, double y, int k);

/* ---- training data of the learned proposal -----------------------------
   All draws use key(seed) and purpose TRAIN.
   Long run q: x_0 ~ tau_0 from counters (q, RUN, 0xFFFFFFFF, s/4) lane s%4;
     Euler step n = 0 .. run_len*S - 1 from counters (q, RUN, n, sub-block of
     the model's layout); start state j of run q is x_{(j+1)S}.
   Trajectory r (start x_0 = start state r): step k = 0 .. S-1 from counters
     (r, TRAJ, k, ...); y_r = H x_S + obs_sd eta, eta_o from counters
     (r, TRAJ, 0xFFFFFFFF, o/4) lane o%4.
   Regression row (r, k, node): features of x_k of trajectory r with y_r at
     step k; target (sd/sqrt(h)) z_k of the node's v and w.
   Minibatch of Adam step s: tile b (16 consecutive nodes) from the words
     (w0, w1, w2) of counter (b, BATCH, s, TRAIN << 24): r = floor(w0 n_traj
     / 2^32), k = w1 mod S, first node 16 floor(w2 (J*J/16) / 2^32). */
#define OR_TRAIN_RUN 0xFFFFFFFEu
#define OR_TRAIN_TRAJ 0xFFFFFFFDu
#define OR_TRAIN_BATCH 0xFFFFFFFCu
void or_train_run(const or_model *m, uint64_t seed, uint32_t q, int run_len,
                  double *starts /* [run_len][dx] */);
void or_train_trajectory(const or_model *m, uint64_t seed, uint32_t r,
                         const double *x0, double *traj /* [S][dx] */,
                         double *y /* [dy] */, double *z /* [S][dx] or NULL */);
void or_train_tile(const or_model *m, uint64_t seed, int n_traj, int step, uint32_t b,
                   int *r, int *k, int *node0);
/* Adam (Kingma and Ba, Alg. 1) on n parameters at step t >= 1 (bias
   corrections 1 - beta^t). */
void or_adam_step(int n, double *p, const double *g, double *mo, double *ve,
                  double lr, double beta1, double beta2, double eps, int t);

#ifdef __cplusplus
}
#endif
#endif
