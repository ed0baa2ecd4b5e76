/*
 * pf_oracle.c -- FP64 single-threaded reference of the independent-ensemble
 * bootstrap particle filter.  TEST INFRASTRUCTURE ONLY (see pf_oracle.h).
 *
 * Every function follows the paper's definition step by step, in the paper's
 * order; nothing is blocked, fused or reordered.
 *
 * Random-number layout (the one contract the GPU side implements again on its
 * own):
 *   key      = (low 32 bits of seed, high 32 bits of seed XOR 0x14078071)
 *   counter  = (c0, c1, c2, c3) with c3 = purpose << 24 | sub-block
 *   uniform  u = (2*(x >> 9) + 1) * 2^-24, exactly representable in FP32
 *   normals  Box-Muller on (u0,u1) -> z0 = r cos(2 pi u1), z1 = r sin(2 pi u1)
 *            with r = sqrt(-2 ln u0); (u2,u3) -> z2, z3 likewise
 *   Euler noise of a particle (c0 = particle, c1 = filter), step n:
 *     vector models of dimension d: c2 = n/4, component c of step n uses
 *       normal l = (n%4)*d + c, i.e. sub-block l/4, lane l%4;
 *     grid model: c2 = n, sub-block p = node/2; lanes 0,1 are the (v, w)
 *       noise of node 2p and lanes 2,3 those of node 2p+1 (nodes row-major);
 *   prior draw: state index s uses c2 = 0, sub-block s/4, lane s%4;
 *   resampling: exponential E_j (j = 0..N) uses c0 = j/4, c1 = filter,
 *     c2 = t, sub-block 0, lane j%4;
 *   truth path: c0 = 0, c1 = 0xFFFFFFFF, purposes TRUTH_INIT / TRUTH_NOISE;
 *   observation noise of y_t component k: c0 = 0, c1 = 0xFFFFFFFF, c2 = t,
 *     sub-block k/4, lane k%4.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): two 32x32->64 multiplications per
   round with the published multipliers, the Weyl key schedule with the
   published increments, ten rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_key(uint64_t seed, uint32_t key[2]) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32) ^ 0x14078071u;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_u01(uint32_t x) {
  return (double)(2u * (x >> 9) + 1u) * 0x1p-24;
}

void or_normals4(const uint32_t ctr[4], const uint32_t key[2], double z[4]) {
  uint32_t r[4];
  or_philox4x32_10(ctr, key, r);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < 4; k += 2) {
    double u0 = or_u01(r[k]);
    double u1 = or_u01(r[k + 1]);
    double rad = sqrt(-2.0 * log(u0));
    z[k] = rad * cos(two_pi * u1);
    z[k + 1] = rad * sin(two_pi * u1);
  }
}

static void make_ctr(uint32_t c[4], uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t purpose, uint32_t sub) {
  c[0] = c0; c[1] = c1; c[2] = c2; c[3] = (purpose << 24) | (sub & 0xFFFFFFu);
}

void or_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, uint32_t *out) {
  uint32_t key[2], ctr[4], r[4];
  or_key(seed, key);
  for (int64_t i = 0; i < n; i += 4) {
    ctr[0] = (uint32_t)(i / 4); ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    or_philox4x32_10(ctr, key, r);
    for (int l = 0; l < 4 && i + l < n; ++l) out[i + l] = r[l];
  }
}

void or_normal_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, double *out) {
  uint32_t key[2], ctr[4];
  double z[4];
  or_key(seed, key);
  for (int64_t i = 0; i < n; i += 4) {
    ctr[0] = (uint32_t)(i / 4); ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    or_normals4(ctr, key, z);
    for (int l = 0; l < 4 && i + l < n; ++l) out[i + l] = z[l];
  }
}

/* ------------------------------------------------------------------------ */
/* Models. */

/* Discrete Laplacian with the truncated neighbourhoods of Sec. 5.2: every
   node is coupled to its up/down/left/right neighbours that exist in the
   grid (two at corners, three on sides, four inside):
   lap_ij = sum_{nbr} (v_nbr - v_ij). */
void or_laplacian(int J, const double *v, double *lap) {
  for (int i = 0; i < J; ++i) {
    for (int j = 0; j < J; ++j) {
      double c = v[i * J + j];
      double acc = 0.0;
      if (i > 0) acc += v[(i - 1) * J + j] - c;
      if (i < J - 1) acc += v[(i + 1) * J + j] - c;
      if (j > 0) acc += v[i * J + j - 1] - c;
      if (j < J - 1) acc += v[i * J + j + 1] - c;
      lap[i * J + j] = acc;
    }
  }
}

void or_drift(const or_model *m, const double *x, double *f) {
  if (m->kind == OR_OU1D) {
    f[0] = -m->p[0] * x[0];
  } else if (m->kind == OR_LORENZ63) {
    /* eqs. (eqDiscreteLorenz-1..3): s(x2 - x1), r x1 - x2 - x1 x3,
       x1 x2 - b x3 */
    double s = m->p[0], r = m->p[1], b = m->p[2];
    f[0] = s * (x[1] - x[0]);
    f[1] = r * x[0] - x[1] - x[0] * x[2];
    f[2] = x[0] * x[1] - b * x[2];
  } else {
    /* FitzHugh-Nagumo grid: v plane x[0..J*J), w plane x[J*J..2J*J).
       f_v = v (v - a)(1 - v) - w + D lap(v), f_w = eps (v - gam w). */
    int J = m->J, nn = J * J;
    double a = m->p[0], D = m->p[1], eps = m->p[2], gam = m->p[3];
    const double *v = x, *w = x + nn;
    double *lap = (double *)malloc(sizeof(double) * (size_t)nn);
    or_laplacian(J, v, lap);
    for (int k = 0; k < nn; ++k) {
      f[k] = v[k] * (v[k] - a) * (1.0 - v[k]) - w[k] + D * lap[k];
      f[nn + k] = eps * (v[k] - gam * w[k]);
    }
    free(lap);
  }
}

void or_step_noise(const or_model *m, const uint32_t key[2], uint32_t purpose,
                   uint32_t c0, uint32_t c1, uint32_t n, double *z) {
  uint32_t ctr[4];
  double q[4];
  if (m->kind == OR_FHN || m->kind == OR_FHN_PAPER) {
    int nn = m->J * m->J;
    for (int p = 0; 2 * p < nn; ++p) {
      make_ctr(ctr, c0, c1, n, purpose, (uint32_t)p);
      or_normals4(ctr, key, q);
      z[2 * p] = q[0];
      z[nn + 2 * p] = q[1];
      if (2 * p + 1 < nn) {
        z[2 * p + 1] = q[2];
        z[nn + 2 * p + 1] = q[3];
      }
    }
  } else {
    int d = m->dx;
    uint32_t r = n % 4u;
    for (int c = 0; c < d; ++c) {
      uint32_t l = r * (uint32_t)d + (uint32_t)c;
      make_ctr(ctr, c0, c1, n / 4u, purpose, l / 4u);
      or_normals4(ctr, key, q);
      z[c] = q[l % 4u];
    }
  }
}

/* ---- the paper's modified FH-N network (Sec. 5.1, 5.2) ------------------ */

/* 4-neighbours of node k inside the grid; returns how many */
static int grid_nbrs(int J, int k, int *nb) {
  int i = k / J, j = k % J, c = 0;
  if (i > 0) nb[c++] = k - J;
  if (i < J - 1) nb[c++] = k + J;
  if (j > 0) nb[c++] = k - 1;
  if (j < J - 1) nb[c++] = k + 1;
  return c;
}

int or_fhnp_region(const or_model *m, const double *U, int *region) {
  int J = m->J, nn = J * J, count = 0, nb[4];
  double lo = m->q[3], hi = m->q[4];
  for (int k = 0; k < nn; ++k) {
    int in = U[k] > lo && U[k] < hi;
    int c = grid_nbrs(J, k, nb);
    for (int e = 0; e < c && !in; ++e) in = U[nb[e]] > lo && U[nb[e]] < hi;
    region[k] = in;
    count += in;
  }
  return count;
}

static int fhnp_step(const or_model *m, const uint32_t key[2], uint32_t purpose, uint32_t c0,
                     uint32_t c1, uint32_t n, const double *x, double *xo, int pilot) {
  int J = m->J, nn = J * J, nb[4];
  int l0 = (int)m->q[5];
  const double *U = x, *V = x + nn;
  double a2 = m->p[0], cpl = m->p[1], b0 = m->p[2], b1 = m->p[3], b2 = m->q[0];
  double amp = m->q[1], eps = m->q[2];
  int *region = (int *)malloc(sizeof(int) * (size_t)nn);
  double *z = (double *)malloc(sizeof(double) * (size_t)m->dx);
  /* 1.-2. stimulus region, Bernoulli event and its centre */
  int count = or_fhnp_region(m, U, region);
  uint32_t ctr[4], r[4];
  make_ctr(ctr, c0, c1, n, purpose, (uint32_t)(nn / 2));
  or_philox4x32_10(ctr, key, r);
  int event = -1;
  if (!pilot && count > 0 && or_u01(r[0]) < eps) {
    int kth = (int)floor(or_u01(r[1]) * (double)count);
    if (kth > count - 1) kth = count - 1;
    for (int k = 0; k < nn; ++k)
      if (region[k] && kth-- == 0) {
        event = k;
        break;
      }
  }
  /* 3. the event history */
  memcpy(xo + 2 * nn, x + 2 * nn, sizeof(double) * (size_t)(m->dx - 2 * nn));
  xo[2 * nn + (int)(n % (uint32_t)l0)] = (double)event;
  /* 4.-6. stimulus, forcing and the Euler step */
  if (pilot)
    memset(z, 0, sizeof(double) * (size_t)m->dx);
  else
    or_step_noise(m, key, purpose, c0, c1, n, z);
  double sq0 = m->sd[0] * sqrt(m->h), sq1 = m->sd[1] * sqrt(m->h);
  int forcing = (int)(n % (uint32_t)m->q[6]) < (int)m->q[7];
  for (int k = 0; k < nn; ++k) {
    int c = grid_nbrs(J, k, nb);
    double sum = 0.0;
    for (int e = 0; e < c; ++e) sum += U[nb[e]];
    int covered = 0;
    for (int l = 0; l < l0 && !covered; ++l) {
      int ev = (int)xo[2 * nn + l];
      if (ev < 0) continue;
      covered = ev == k;
      int cn = grid_nbrs(J, ev, nb);
      for (int e = 0; e < cn && !covered; ++e) covered = nb[e] == k;
    }
    double psi = covered ? amp : 0.0;
    double mf = (forcing && k / J < 2 && k % J < 2) ? amp : 0.0;
    double u = U[k], v = V[k];
    double p3 = a2 * u - u * u * u;
    xo[k] = ((u + m->h * (p3 - v)) + m->h * (cpl * sum + mf + psi)) + sq0 * z[k];
    xo[nn + k] = (v + m->h * (b0 * u + b1 * v + b2)) + sq1 * z[nn + k];
  }
  free(region);
  free(z);
  return event;
}

int or_fhnp_step(const or_model *m, const uint32_t key[2], uint32_t purpose, uint32_t c0,
                 uint32_t c1, uint32_t n, const double *x, double *xo) {
  return fhnp_step(m, key, purpose, c0, c1, n, x, xo, 0);
}

/* The noise-free continuation of one step: no new stimulus event (the
   ring's active stimuli and the forcing still act) and no noise. */
void or_pilot_step(const or_model *m, uint32_t n, const double *x, double *xo) {
  if (m->kind == OR_FHN_PAPER) {
    uint32_t key[2] = {0u, 0u};
    fhnp_step(m, key, 0u, 0u, 0u, n, x, xo, 1);
    return;
  }
  double *z = (double *)calloc((size_t)m->dx, sizeof(double));
  or_em_step(m, x, z, xo);
  free(z);
}

/* Euler-Maruyama: x' = x + h f(x) + sd sqrt(h) z (drift first, then the
   deterministic update, then the noise). */
void or_em_step(const or_model *m, const double *x, const double *z, double *xo) {
  int d = m->dx;
  double *f = (double *)malloc(sizeof(double) * (size_t)d);
  or_drift(m, x, f);
  double sq0 = m->sd[0] * sqrt(m->h);
  double sq1 = m->sd[1] * sqrt(m->h);
  int half = (m->kind == OR_FHN) ? m->J * m->J : d;
  for (int k = 0; k < d; ++k) {
    double sq = (k < half) ? sq0 : sq1;
    xo[k] = (x[k] + m->h * f[k]) + sq * z[k];
  }
  free(f);
}

void or_transition(const or_model *m, const uint32_t key[2], uint32_t purpose, uint32_t c0,
                   uint32_t c1, uint32_t n, const double *x, double *xo) {
  if (m->kind == OR_FHN_PAPER) {
    or_fhnp_step(m, key, purpose, c0, c1, n, x, xo);
    return;
  }
  double *z = (double *)malloc(sizeof(double) * (size_t)m->dx);
  or_step_noise(m, key, purpose, c0, c1, n, z);
  or_em_step(m, x, z, xo);
  free(z);
}

void or_prior_draw(const or_model *m, const uint32_t key[2], uint32_t purpose,
                   uint32_t c0, uint32_t c1, double *x) {
  uint32_t ctr[4];
  double q[4];
  for (int s = 0; s < m->dx; s += 4) {
    make_ctr(ctr, c0, c1, 0u, purpose, (uint32_t)(s / 4));
    or_normals4(ctr, key, q);
    for (int l = 0; l < 4 && s + l < m->dx; ++l)
      x[s + l] = m->prior_mean[s + l] + m->prior_sd[s + l] * q[l];
  }
}

/* log g_t^{y}(x) up to the additive constant: -(1/(2 sigma^2)) sum (y-Hx)^2
   (eqObservLorenz likelihood, eqObservFHN likelihood).  A NaN state gives
   -inf (the particle can never be selected). */
double or_loglik(const or_model *m, const double *x, const double *y) {
  double acc = 0.0;
  for (int k = 0; k < m->dy; ++k) {
    double r = y[k] - x[m->obs_idx[k]];
    acc += r * r;
  }
  double lw = -acc / (2.0 * m->obs_var);
  if (isnan(lw)) lw = -INFINITY;
  return lw;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, one filter. */

/* Step 1: x_0^(i) ~ tau_0, i = 1..N. */
void or_init(const or_model *m, uint64_t seed, uint32_t filter, int N, double *X) {
  uint32_t key[2];
  or_key(seed, key);
  for (int i = 0; i < N; ++i)
    or_prior_draw(m, key, OR_P_INIT, (uint32_t)i, filter, X + (size_t)i * m->dx);
}

/* Step 2(a), sampling: xbar_t^(i) ~ tau_t(.|x_{t-1}^(i)), realised as S
   Euler-Maruyama steps n = (t-1)S .. tS-1 (Sec. 4.1). */
void or_propagate(const or_model *m, uint64_t seed, uint32_t filter, int N,
                  int t, double *X) {
  uint32_t key[2];
  or_key(seed, key);
  int d = m->dx;
  double *xn = (double *)malloc(sizeof(double) * (size_t)d);
  for (int i = 0; i < N; ++i) {
    double *x = X + (size_t)i * d;
    for (int s = 0; s < m->S; ++s) {
      uint32_t n = (uint32_t)((t - 1) * m->S + s);
      or_transition(m, key, OR_P_PROP, (uint32_t)i, filter, n, x, xn);
      memcpy(x, xn, sizeof(double) * (size_t)d);
    }
  }
  free(xn);
}

/* The same draw for one particle of index `index` (Philox counter word 0),
   so that a sample of a large filter can be checked particle by particle. */
void or_propagate_particle(const or_model *m, uint64_t seed, uint32_t filter,
                           uint32_t index, int t, double *x) {
  uint32_t key[2];
  or_key(seed, key);
  int d = m->dx;
  double *xn = (double *)malloc(sizeof(double) * (size_t)d);
  for (int s = 0; s < m->S; ++s) {
    uint32_t n = (uint32_t)((t - 1) * m->S + s);
    or_transition(m, key, OR_P_PROP, index, filter, n, x, xn);
    memcpy(x, xn, sizeof(double) * (size_t)d);
  }
  free(xn);
}

/* Step 2(a), weighting: log g_t^{y_t}(xbar_t^(i)). */
void or_weights(const or_model *m, int N, const double *X, const double *y,
                double *lw) {
  for (int i = 0; i < N; ++i) lw[i] = or_loglik(m, X + (size_t)i * m->dx, y);
}

/* Step 2(a), normalisation: w^(i) = g(xbar^(i)) / sum_k g(xbar^(k)), carried
   as mx = max lw and W = sum exp(lw - mx) (sequential, index order).  If no
   weight is positive the weights are taken as uniform and 1 is returned. */
int or_normalise(int N, const double *lw, double *mx, double *W, double *sumw2) {
  double m = -INFINITY;
  for (int i = 0; i < N; ++i)
    if (lw[i] > m) m = lw[i];
  if (!(m > -INFINITY) || isnan(m) || isinf(m)) {
    *mx = -INFINITY;
    *W = (double)N;
    *sumw2 = (double)N;
    return 1;
  }
  double s = 0.0, s2 = 0.0;
  for (int i = 0; i < N; ++i) {
    double w = exp(lw[i] - m);
    s += w;
    s2 += w * w;
  }
  *mx = m;
  *W = s;
  *sumw2 = s2;
  return 0;
}

/* Effective sample size of the normalised weights, (sum w)^2 / sum w^2
   (N when no weight is positive: the weights are then taken as uniform). */
double or_ess(int N, const double *lw) {
  double mx, W, s2;
  or_normalise(N, lw, &mx, &W, &s2);
  return W * W / s2;
}

/* Cumulative weights C_i = sum_{j<=i} exp(lw_j - mx) (uniform if degenerate). */
void or_cdf(int N, const double *lw, double mx, int degenerate, double *C) {
  double acc = 0.0;
  for (int i = 0; i < N; ++i) {
    acc += degenerate ? 1.0 : exp(lw[i] - mx);
    C[i] = acc;
  }
}

/* Sorted uniforms by exponential spacings (Devroye 1986, Ch. V.3):
   E_j = -ln u_j, j = 0..N; S_k = sum_{j<=k} E_j; U_k = S_k / S_N for
   k = 0..N-1 are the order statistics of N independent U(0,1). */
void or_sorted_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U) {
  uint32_t key[2], ctr[4], r[4];
  or_key(seed, key);
  double *S = (double *)malloc(sizeof(double) * (size_t)(N + 1));
  double acc = 0.0;
  for (int j = 0; j <= N; ++j) {
    if (j % 4 == 0) {
      make_ctr(ctr, (uint32_t)(j / 4), filter, (uint32_t)t, OR_P_RESAMPLE, 0u);
      or_philox4x32_10(ctr, key, r);
    }
    acc += -log(or_u01(r[j % 4]));
    S[j] = acc;
  }
  for (int k = 0; k < N; ++k) U[k] = S[k] / S[N];
  free(S);
}

/* Step 2(b), multinomial selection: ancestor a_k = min{ i : C_i > U_k C_{N-1} }
   for the ascending U, found with one forward pointer over C. */
void or_ancestors(int N, const double *C, const double *U, int32_t *A) {
  int i = 0;
  double total = C[N - 1];
  for (int k = 0; k < N; ++k) {
    double v = U[k] * total;
    while (i < N - 1 && C[i] <= v) ++i;
    A[k] = i;
  }
}

void or_gather(int N, int dx, const double *X, const int32_t *A, double *Xo) {
  for (int k = 0; k < N; ++k)
    memcpy(Xo + (size_t)k * dx, X + (size_t)A[k] * dx, sizeof(double) * (size_t)dx);
}

/* (f, pi_t^N) with f the identity: (1/N) sum_i x_t^(i). */
void or_mean(int N, int dx, const double *X, double *mean) {
  for (int c = 0; c < dx; ++c) mean[c] = 0.0;
  for (int i = 0; i < N; ++i)
    for (int c = 0; c < dx; ++c) mean[c] += X[(size_t)i * dx + c];
  for (int c = 0; c < dx; ++c) mean[c] /= (double)N;
}

/* sum_i w^(i) xbar^(i): the weighted (pre-resampling) estimate. */
void or_weighted_mean(int N, int dx, const double *X, const double *lw,
                      double mx, double *mean) {
  double W = 0.0;
  for (int c = 0; c < dx; ++c) mean[c] = 0.0;
  int degenerate = !(mx > -INFINITY);
  for (int i = 0; i < N; ++i) {
    double w = degenerate ? 1.0 : exp(lw[i] - mx);
    W += w;
    for (int c = 0; c < dx; ++c) mean[c] += w * X[(size_t)i * dx + c];
  }
  for (int c = 0; c < dx; ++c) mean[c] /= W;
}

int or_filter_interval(const or_model *m, uint64_t seed, uint32_t filter, int N,
                       int t, double *X, const double *y, double *logZ,
                       double *lw_out, int32_t *A_out, double *mean_post,
                       double *mean_w, double *ess) {
  int d = m->dx;
  double *lw = (double *)malloc(sizeof(double) * (size_t)N);
  double *C = (double *)malloc(sizeof(double) * (size_t)N);
  double *U = (double *)malloc(sizeof(double) * (size_t)N);
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *Xo = (double *)malloc(sizeof(double) * (size_t)N * d);
  double mx, W, s2;

  or_propagate(m, seed, filter, N, t, X);
  or_weights(m, N, X, y, lw);
  int deg = or_normalise(N, lw, &mx, &W, &s2);
  if (logZ) {
    const double two_pi = 6.283185307179586476925286766559;
    if (deg)
      *logZ = -INFINITY;
    else
      *logZ += mx + log(W / (double)N) - 0.5 * m->dy * log(two_pi * m->obs_var);
  }
  if (ess) *ess = W * W / s2;
  if (mean_w) or_weighted_mean(N, d, X, lw, mx, mean_w);
  or_cdf(N, lw, mx, deg, C);
  or_sorted_uniforms(seed, filter, t, N, U);
  or_ancestors(N, C, U, A);
  or_gather(N, d, X, A, Xo);
  memcpy(X, Xo, sizeof(double) * (size_t)N * d);
  if (mean_post) or_mean(N, d, X, mean_post);
  if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)N);
  if (A_out) memcpy(A_out, A, sizeof(int32_t) * (size_t)N);
  free(lw); free(C); free(U); free(A); free(Xo);
  return deg;
}

/* ------------------------------------------------------------------------ */
/* Other resampling schemes (Sec. 2.3) and the ESS-triggered schedule.       */

static double rs_uniform(const uint32_t key[2], uint32_t c0, uint32_t filter, int t,
                         uint32_t sub, int lane) {
  uint32_t ctr[4], r[4];
  make_ctr(ctr, c0, filter, (uint32_t)t, OR_P_RESAMPLE, sub);
  or_philox4x32_10(ctr, key, r);
  return or_u01(r[lane]);
}

/* Systematic resampling: the N points share one uniform offset. */
void or_systematic_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U) {
  uint32_t key[2];
  or_key(seed, key);
  double u = rs_uniform(key, 0u, filter, t, 1u, 0);
  for (int k = 0; k < N; ++k) U[k] = ((double)k + u) / (double)N;
}

/* Stratified resampling: one uniform point in each stratum [k/N, (k+1)/N). */
void or_stratified_uniforms(uint64_t seed, uint32_t filter, int t, int N, double *U) {
  uint32_t key[2];
  or_key(seed, key);
  for (int k = 0; k < N; ++k) {
    double u = rs_uniform(key, (uint32_t)(k / 4), filter, t, 2u, k % 4);
    U[k] = ((double)k + u) / (double)N;
  }
}

/* Residual resampling: the integer parts of N w_i / W deterministically,
   the remainder multinomially from the fractional parts. */
void or_residual_ancestors(uint64_t seed, uint32_t filter, int t, int N, const double *lw,
                           double mx, int degenerate, int32_t *A) {
  double *w = (double *)malloc(sizeof(double) * (size_t)N);
  double *Cr = (double *)malloc(sizeof(double) * (size_t)N);
  int *cnt = (int *)malloc(sizeof(int) * (size_t)N);
  double W = 0.0;
  for (int i = 0; i < N; ++i) {
    w[i] = degenerate ? 1.0 : exp(lw[i] - mx);
    W += w[i];
  }
  int R = N;
  double acc = 0.0;
  for (int i = 0; i < N; ++i) {
    double nw = (double)N * w[i] / W;
    double fl = floor(nw);
    cnt[i] = (int)fl;
    R -= cnt[i];
    acc += nw - fl;
    Cr[i] = acc;
  }
  if (R > 0) {
    /* R sorted uniforms from the spacings of R + 1 exponentials */
    uint32_t key[2], ctr[4], r[4];
    or_key(seed, key);
    double *S = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    double s = 0.0;
    for (int j = 0; j <= R; ++j) {
      if (j % 4 == 0) {
        make_ctr(ctr, (uint32_t)(j / 4), filter, (uint32_t)t, OR_P_RESAMPLE, 0u);
        or_philox4x32_10(ctr, key, r);
      }
      s += -log(or_u01(r[j % 4]));
      S[j] = s;
    }
    int i = 0;
    for (int k = 0; k < R; ++k) {
      double v = (S[k] / S[R]) * Cr[N - 1];
      while (i < N - 1 && Cr[i] <= v) ++i;
      cnt[i] += 1;
    }
    free(S);
  }
  int k = 0;
  for (int i = 0; i < N; ++i)
    for (int c = 0; c < cnt[i]; ++c) A[k++] = i;
  free(w); free(Cr); free(cnt);
}

void or_resample_scheme(int scheme, uint64_t seed, uint32_t filter, int t, int N,
                        const double *lw, int32_t *A) {
  double mx, W, s2;
  int deg = or_normalise(N, lw, &mx, &W, &s2);
  if (scheme == OR_RS_RESIDUAL) {
    or_residual_ancestors(seed, filter, t, N, lw, mx, deg, A);
    return;
  }
  double *C = (double *)malloc(sizeof(double) * (size_t)N);
  double *U = (double *)malloc(sizeof(double) * (size_t)N);
  or_cdf(N, lw, mx, deg, C);
  if (scheme == OR_RS_SYSTEMATIC)
    or_systematic_uniforms(seed, filter, t, N, U);
  else if (scheme == OR_RS_STRATIFIED)
    or_stratified_uniforms(seed, filter, t, N, U);
  else
    or_sorted_uniforms(seed, filter, t, N, U);
  or_ancestors(N, C, U, A);
  free(C); free(U);
}

int or_filter_interval_sched(const or_model *m, uint64_t seed, uint32_t filter, int N, int t,
                             double *X, double *lwc, const double *y, double *logZ, int scheme,
                             double ess_threshold, double *lw_out, int32_t *A_out,
                             double *mean_est, double *mean_w, double *ess_out,
                             int *resampled_out) {
  int d = m->dx;
  double *lw = (double *)malloc(sizeof(double) * (size_t)N);
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *Xo = (double *)malloc(sizeof(double) * (size_t)N * d);
  double mx, W, s2;

  or_propagate(m, seed, filter, N, t, X);
  or_weights(m, N, X, y, lw);
  for (int i = 0; i < N; ++i) lw[i] += lwc[i];
  int deg = or_normalise(N, lw, &mx, &W, &s2);
  if (logZ) {
    const double two_pi = 6.283185307179586476925286766559;
    if (deg)
      *logZ = -INFINITY;
    else
      *logZ += mx + log(W / (double)N) - 0.5 * m->dy * log(two_pi * m->obs_var);
  }
  double ess = W * W / s2;
  if (ess_out) *ess_out = ess;
  if (mean_w) or_weighted_mean(N, d, X, lw, mx, mean_w);
  int resample = deg || ess_threshold <= 0.0 || ess < ess_threshold * (double)N;
  if (resample) {
    or_resample_scheme(scheme, seed, filter, t, N, lw, A);
    or_gather(N, d, X, A, Xo);
    memcpy(X, Xo, sizeof(double) * (size_t)N * d);
    for (int i = 0; i < N; ++i) lwc[i] = 0.0;
    if (mean_est) or_mean(N, d, X, mean_est);
  } else {
    double shift = mx + log(W / (double)N);
    for (int i = 0; i < N; ++i) {
      A[i] = i;
      lwc[i] = lw[i] - shift;
    }
    if (mean_est) or_weighted_mean(N, d, X, lw, mx, mean_est);
  }
  if (resampled_out) *resampled_out = resample;
  if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)N);
  if (A_out) memcpy(A_out, A, sizeof(int32_t) * (size_t)N);
  free(lw); free(A); free(Xo);
  return deg;
}

int or_apf_interval(const or_model *m, uint64_t seed, uint32_t filter, int N, int t, double *X,
                    double *lwc, const double *y, double *logZ, int scheme, double *lw_out,
                    int32_t *A_out, double *mean_w, double *ess_out) {
  const double two_pi = 6.283185307179586476925286766559;
  int d = m->dx;
  double *pil = (double *)calloc((size_t)N, sizeof(double));
  double *lam = (double *)calloc((size_t)N, sizeof(double));
  double *lw = (double *)malloc(sizeof(double) * (size_t)N);
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *Xo = (double *)malloc(sizeof(double) * (size_t)N * d);
  double *mu = (double *)malloc(sizeof(double) * (size_t)d);
  double *nx = (double *)malloc(sizeof(double) * (size_t)d);
  double mx, W, s2;
  /* 1. the pilot: noise-free Euler path and its likelihood */
  for (int i = 0; i < N; ++i) {
    memcpy(mu, X + (size_t)i * d, sizeof(double) * (size_t)d);
    for (int s = 0; s < m->S; ++s) {
      or_pilot_step(m, (uint32_t)((t - 1) * m->S + s), mu, nx);
      memcpy(mu, nx, sizeof(double) * (size_t)d);
    }
    pil[i] = or_loglik(m, mu, y);
    lam[i] = lwc[i] + pil[i];
  }
  /* 2. first-stage resampling */
  int deg1 = or_normalise(N, lam, &mx, &W, &s2);
  double lz1 = deg1 ? -INFINITY : mx + log(W / (double)N);
  or_resample_scheme(scheme, seed, filter, t, N, lam, A);
  /* 3. propagation of the selected particles, slot k */
  or_gather(N, d, X, A, Xo);
  or_propagate(m, seed, filter, N, t, Xo);
  memcpy(X, Xo, sizeof(double) * (size_t)N * d);
  /* 4. second-stage weights, carried */
  or_weights(m, N, X, y, lw);
  for (int k = 0; k < N; ++k) lw[k] -= pil[A[k]];
  int deg2 = or_normalise(N, lw, &mx, &W, &s2);
  if (logZ) {
    if (deg1 || deg2)
      *logZ = -INFINITY;
    else
      *logZ += lz1 + mx + log(W / (double)N) - 0.5 * m->dy * log(two_pi * m->obs_var);
  }
  if (ess_out) *ess_out = W * W / s2;
  if (mean_w) or_weighted_mean(N, d, X, lw, mx, mean_w);
  for (int k = 0; k < N; ++k) lwc[k] = deg2 ? 0.0 : lw[k] - (mx + log(W / (double)N));
  if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)N);
  if (A_out) memcpy(A_out, A, sizeof(int32_t) * (size_t)N);
  free(pil); free(lam); free(lw); free(A); free(Xo); free(mu); free(nx);
  return deg1 || deg2;
}

/* Definition 3: M independent filters on the same y_{1:T}, averaged with
   equal weights 1/M. */
void or_run_ensemble(const or_model *m, uint64_t seed, int M, int N, int T,
                     const double *y, double *est, double *est_w,
                     double *logZ, double *ess) {
  int d = m->dx;
  double *X = (double *)malloc(sizeof(double) * (size_t)N * d);
  double *mp = (double *)malloc(sizeof(double) * (size_t)d);
  double *mw = (double *)malloc(sizeof(double) * (size_t)d);
  if (est) memset(est, 0, sizeof(double) * (size_t)T * d);
  if (est_w) memset(est_w, 0, sizeof(double) * (size_t)T * d);
  if (ess) memset(ess, 0, sizeof(double) * (size_t)T);
  for (int f = 0; f < M; ++f) {
    double lz = 0.0;
    or_init(m, seed, (uint32_t)f, N, X);
    for (int t = 1; t <= T; ++t) {
      double e;
      or_filter_interval(m, seed, (uint32_t)f, N, t, X, y + (size_t)(t - 1) * m->dy,
                         &lz, NULL, NULL, mp, mw, &e);
      for (int c = 0; c < d; ++c) {
        if (est) est[(size_t)(t - 1) * d + c] += mp[c] / (double)M;
        if (est_w) est_w[(size_t)(t - 1) * d + c] += mw[c] / (double)M;
      }
      if (ess) ess[t - 1] += e / (double)M;
    }
    if (logZ) logZ[f] = lz;
  }
  free(X); free(mp); free(mw);
}

void or_simulate(const or_model *m, uint64_t seed, int T, double *x_true,
                 double *y) {
  uint32_t key[2], ctr[4];
  double q[4];
  int d = m->dx;
  or_key(seed, key);
  double *x = (double *)malloc(sizeof(double) * (size_t)d);
  double *z = (double *)malloc(sizeof(double) * (size_t)d);
  double *xn = (double *)malloc(sizeof(double) * (size_t)d);
  or_prior_draw(m, key, OR_P_TRUTH_INIT, 0u, OR_TRUTH_STREAM, x);
  memcpy(x_true, x, sizeof(double) * (size_t)d);
  double sy = sqrt(m->obs_var);
  for (int t = 1; t <= T; ++t) {
    for (int s = 0; s < m->S; ++s) {
      uint32_t n = (uint32_t)((t - 1) * m->S + s);
      or_transition(m, key, OR_P_TRUTH_NOISE, 0u, OR_TRUTH_STREAM, n, x, xn);
      memcpy(x, xn, sizeof(double) * (size_t)d);
    }
    memcpy(x_true + (size_t)t * d, x, sizeof(double) * (size_t)d);
    for (int k = 0; k < m->dy; k += 4) {
      make_ctr(ctr, 0u, OR_TRUTH_STREAM, (uint32_t)t, OR_P_OBS_NOISE, (uint32_t)(k / 4));
      or_normals4(ctr, key, q);
      for (int l = 0; l < 4 && k + l < m->dy; ++l)
        y[(size_t)(t - 1) * m->dy + k + l] = x[m->obs_idx[k + l]] + sy * q[l];
    }
  }
  free(x); free(z); free(xn);
}

/* Exact filter for x_{n+1} = (1 - theta h) x_n + sd sqrt(h) z observed as
   y_t = x_{tS} + N(0, obs_var): the interval transition is
   x_{tS} = a x_{(t-1)S} + N(0, q) with a = (1-theta h)^S and
   q = sd^2 h sum_{i<S} (1-theta h)^{2i}. */
double or_kalman_ou(const or_model *m, int T, const double *y, double *mean,
                    double *var) {
  double phi = 1.0 - m->p[0] * m->h;
  double a = 1.0, q = 0.0;
  for (int i = 0; i < m->S; ++i) {
    q += m->sd[0] * m->sd[0] * m->h * a * a;
    a *= phi;
  }
  double mu = m->prior_mean[0], P = m->prior_sd[0] * m->prior_sd[0];
  double R = m->obs_var, ll = 0.0;
  const double two_pi = 6.283185307179586476925286766559;
  for (int t = 0; t < T; ++t) {
    double mp = a * mu, Pp = a * a * P + q;
    double Sv = Pp + R;
    double r = y[t] - mp;
    ll += -0.5 * (log(two_pi * Sv) + r * r / Sv);
    double K = Pp / Sv;
    mu = mp + K * r;
    P = (1.0 - K) * Pp;
    if (mean) mean[t] = mu;
    if (var) var[t] = P;
  }
  return ll;
}

/* ------------------------------------------------------------------------ */
/* Learned proposal.  The paper's convergence results hold for any importance
   function whose weights are the exact density ratio (its closing remarks on
   tailored importance functions, Sec. 6); the proposal here is a drift
   correction u added to each Euler-Maruyama increment, and the weight of a
   particle gains, per step and component, the log ratio of the model density
   N(x + h f, sd^2 h) to the proposal density N(x + h f + h u, sd^2 h) at the
   sampled increment.  With x' - x - h f = h u + sd sqrt(h) z the squares
   expand to -(sqrt(h)/sd) u z - (h/(2 sd^2)) u^2. */

int or_mlp_nparams(int in_dim, int out_dim) {
  const int H = OR_MLP_HIDDEN;
  return H * in_dim + H + H * H + H + out_dim * H + out_dim;
}

/* Round to the nearest bfloat16 (8 significant bits), ties to even. */
double or_bf16(double x) {
  if (x == 0.0 || isnan(x) || isinf(x)) return x;
  int e;
  double m = frexp(x, &e);           /* x = m 2^e, 0.5 <= |m| < 1 */
  double r = nearbyint(ldexp(m, 8)); /* 8 significant bits, ties to even */
  return ldexp(r, e - 8);
}

static double relu(double a) { return a > 0.0 ? a : 0.0; }

/* Forward pass; `rin` rounds inputs and hidden activations, `rw` the
   parameters (both 0 in FP64 mode, both 1 in bfloat16 mode; a caller that has
   rounded the parameters once already passes rw = 0, which gives the same
   values since rounding a bfloat16 number returns it unchanged). */
static void mlp_forward(int in_dim, int out_dim, const double *p, const double *x,
                        double *h1_out, double *h2_out, double *out, int rin, int rw) {
  const int H = OR_MLP_HIDDEN;
  const double *W1 = p, *b1 = W1 + H * in_dim, *W2 = b1 + H, *b2 = W2 + H * H;
  const double *W3 = b2 + H, *b3 = W3 + out_dim * H;
  double h1[OR_MLP_HIDDEN], h2[OR_MLP_HIDDEN];
#define QI(v) (rin ? or_bf16(v) : (v))
#define QW(v) (rw ? or_bf16(v) : (v))
  for (int j = 0; j < H; ++j) {
    double a = QW(b1[j]);
    for (int i = 0; i < in_dim; ++i) a += QW(W1[j * in_dim + i]) * QI(x[i]);
    h1[j] = QI(relu(a));
  }
  for (int j = 0; j < H; ++j) {
    double a = QW(b2[j]);
    for (int i = 0; i < H; ++i) a += QW(W2[j * H + i]) * h1[i];
    h2[j] = QI(relu(a));
  }
  for (int c = 0; c < out_dim; ++c) {
    double a = QW(b3[c]);
    for (int i = 0; i < H; ++i) a += QW(W3[c * H + i]) * h2[i];
    out[c] = a;
  }
#undef QI
#undef QW
  if (h1_out) memcpy(h1_out, h1, sizeof h1);
  if (h2_out) memcpy(h2_out, h2, sizeof h2);
}

void or_mlp_forward(int in_dim, int out_dim, const double *p, const double *x,
                    double *h1_out, double *h2_out, double *out, int bf16) {
  mlp_forward(in_dim, out_dim, p, x, h1_out, h2_out, out, bf16, bf16);
}

/* Reverse-mode derivative of dout . out, layer by layer (chain rule; the
   ReLU derivative is taken as 0 at 0). */
void or_mlp_backward(int in_dim, int out_dim, const double *p, const double *x,
                     const double *dout, double *grad) {
  const int H = OR_MLP_HIDDEN;
  const double *W2 = p + H * in_dim + H, *W3 = W2 + H * H + H;
  double *gW1 = grad, *gb1 = gW1 + H * in_dim, *gW2 = gb1 + H, *gb2 = gW2 + H * H;
  double *gW3 = gb2 + H, *gb3 = gW3 + out_dim * H;
  double h1[OR_MLP_HIDDEN], h2[OR_MLP_HIDDEN], o[16];
  double d2[OR_MLP_HIDDEN], d1[OR_MLP_HIDDEN];
  or_mlp_forward(in_dim, out_dim, p, x, h1, h2, o, 0);
  for (int c = 0; c < out_dim; ++c) {
    gb3[c] += dout[c];
    for (int i = 0; i < H; ++i) gW3[c * H + i] += dout[c] * h2[i];
  }
  for (int i = 0; i < H; ++i) {
    double a = 0.0;
    for (int c = 0; c < out_dim; ++c) a += W3[c * H + i] * dout[c];
    d2[i] = h2[i] > 0.0 ? a : 0.0;
  }
  for (int j = 0; j < H; ++j) {
    gb2[j] += d2[j];
    for (int i = 0; i < H; ++i) gW2[j * H + i] += d2[j] * h1[i];
  }
  for (int i = 0; i < H; ++i) {
    double a = 0.0;
    for (int j = 0; j < H; ++j) a += W2[j * H + i] * d2[j];
    d1[i] = h1[i] > 0.0 ? a : 0.0;
  }
  for (int j = 0; j < H; ++j) {
    gb1[j] += d1[j];
    for (int i = 0; i < in_dim; ++i) gW1[j * in_dim + i] += d1[j] * x[i];
  }
}

double or_mlp_loss_grad(int in_dim, int out_dim, const double *p, int B,
                        const double *X, const double *T, double *grad) {
  double o[16], d[16], loss = 0.0;
  if (grad) memset(grad, 0, sizeof(double) * (size_t)or_mlp_nparams(in_dim, out_dim));
  for (int r = 0; r < B; ++r) {
    const double *x = X + (size_t)r * in_dim, *t = T + (size_t)r * out_dim;
    or_mlp_forward(in_dim, out_dim, p, x, NULL, NULL, o, 0);
    for (int c = 0; c < out_dim; ++c) {
      double e = o[c] - t[c];
      loss += e * e;
      d[c] = 2.0 * e / (double)B;
    }
    if (grad) or_mlp_backward(in_dim, out_dim, p, x, d, grad);
  }
  return loss / (double)B;
}

void or_nearest_obs(const or_model *m, int *map) {
  int J = m->J;
  for (int n = 0; n < J * J; ++n) {
    int i = n / J, j = n % J, best = 0;
    long bd = -1;
    for (int o = 0; o < m->dy; ++o) {
      int r = m->obs_idx[o] / J, c = m->obs_idx[o] % J;
      long d = (long)(i - r) * (i - r) + (long)(j - c) * (j - c);
      if (bd < 0 || d < bd) { bd = d; best = o; }
    }
    map[n] = best;
  }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* 22 features of node `node` at step k of the interval: v patch (9), w patch
   (9), residual of the nearest observation, tau = (S - k)/S, and the row and
   column offsets of that observation, halved. */
void or_fhn_features(const or_model *m, const double *x, const double *y,
                     const int *nearest, int k, int node, double *feat) {
  int J = m->J, nn = J * J, i = node / J, j = node % J;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj) {
      int q = clampi(i + di, 0, J - 1) * J + clampi(j + dj, 0, J - 1);
      feat[(di + 1) * 3 + (dj + 1)] = x[q];
      feat[9 + (di + 1) * 3 + (dj + 1)] = x[nn + q];
    }
  int o = nearest[node];
  feat[18] = y[o] - x[m->obs_idx[o]];
  feat[19] = (double)(m->S - k) / (double)m->S;
  feat[20] = 0.5 * (double)(m->obs_idx[o] / J - i);
  feat[21] = 0.5 * (double)(m->obs_idx[o] % J - j);
}

void or_ou_features(const or_model *m, const double *x, const double *y, int k,
                    double *feat) {
  feat[0] = x[0];
  feat[1] = y[0] - x[0];
  feat[2] = (double)(m->S - k) / (double)m->S;
}

/* u_theta for every state component at step k (FHN: out 0 drives v, out 1
   drives w of the node; OU: the single output). */
/* (p is already rounded to bfloat16 in bfloat16 mode) */
static void learned_drift(const or_model *m, const double *p, const double *x,
                          const double *y, const int *nearest, int k, double *u,
                          int bf16) {
  double feat[22], o[2];
  if (m->kind == OR_FHN) {
    int nn = m->J * m->J;
    for (int n = 0; n < nn; ++n) {
      or_fhn_features(m, x, y, nearest, k, n, feat);
      mlp_forward(22, 2, p, feat, NULL, NULL, o, bf16, 0);
      u[n] = o[0];
      u[nn + n] = o[1];
    }
  } else {
    or_ou_features(m, x, y, k, feat);
    mlp_forward(3, 1, p, feat, NULL, NULL, o, bf16, 0);
    u[0] = o[0];
  }
}

/* One particle (Philox counter word 0 = index) through interval t under the
   learned proposal; returns the sum of its log increment-density ratios.
   pr: the parameters (rounded to bfloat16 in bfloat16 mode), nearest: each
   node's nearest observation (FH-N; NULL otherwise). */
static double propagate_learned_one(const or_model *m, const double *pr, const uint32_t key[2],
                                    uint32_t filter, uint32_t index, int t, double *x,
                                    const double *y, const int *nearest, int bf16) {
  int d = m->dx;
  int half = (m->kind == OR_FHN) ? m->J * m->J : d;
  double *z = (double *)malloc(sizeof(double) * (size_t)d);
  double *f = (double *)malloc(sizeof(double) * (size_t)d);
  double *u = (double *)malloc(sizeof(double) * (size_t)d);
  const double sh = sqrt(m->h);
  double acc = 0.0;
  for (int s = 0; s < m->S; ++s) {
    uint32_t n = (uint32_t)((t - 1) * m->S + s);
    or_step_noise(m, key, OR_P_PROP, index, filter, n, z);
    or_drift(m, x, f);
    learned_drift(m, pr, x, y, nearest, s, u, bf16);
    for (int c = 0; c < d; ++c) {
      double sd = (c < half) ? m->sd[0] : m->sd[1];
      x[c] = (x[c] + m->h * (f[c] + u[c])) + sd * sh * z[c];
      acc += -(sh / sd) * u[c] * z[c] - (m->h / (2.0 * sd * sd)) * u[c] * u[c];
    }
  }
  free(z); free(f); free(u);
  return acc;
}

/* The parameters as the network uses them: rounded once in bfloat16 mode. */
static double *learned_params(const or_model *m, const double *p, int bf16) {
  int np = (m->kind == OR_FHN) ? or_mlp_nparams(22, 2) : or_mlp_nparams(3, 1);
  double *pr = (double *)malloc(sizeof(double) * (size_t)np);
  for (int i = 0; i < np; ++i) pr[i] = bf16 ? or_bf16(p[i]) : p[i];
  return pr;
}

void or_propagate_learned(const or_model *m, const double *p, uint64_t seed,
                          uint32_t filter, int N, int t, double *X,
                          const double *y, double *dlw, int bf16) {
  uint32_t key[2];
  or_key(seed, key);
  int *nearest = NULL;
  if (m->kind == OR_FHN) {
    nearest = (int *)malloc(sizeof(int) * (size_t)(m->J * m->J));
    or_nearest_obs(m, nearest);
  }
  double *pr = learned_params(m, p, bf16);
  for (int i = 0; i < N; ++i)
    dlw[i] = propagate_learned_one(m, pr, key, filter, (uint32_t)i, t, X + (size_t)i * m->dx, y,
                                   nearest, bf16);
  free(pr); free(nearest);
}

double or_propagate_learned_particle(const or_model *m, const double *p, uint64_t seed,
                                     uint32_t filter, uint32_t index, int t, double *x,
                                     const double *y, int bf16) {
  uint32_t key[2];
  or_key(seed, key);
  int *nearest = NULL;
  if (m->kind == OR_FHN) {
    nearest = (int *)malloc(sizeof(int) * (size_t)(m->J * m->J));
    or_nearest_obs(m, nearest);
  }
  double *pr = learned_params(m, p, bf16);
  double r = propagate_learned_one(m, pr, key, filter, index, t, x, y, nearest, bf16);
  free(pr); free(nearest);
  return r;
}

int or_filter_interval_learned(const or_model *m, const double *p, uint64_t seed,
                               uint32_t filter, int N, int t, double *X,
                               const double *y, double *logZ, double *lw_out,
                               int32_t *A_out, double *mean_post, double *mean_w,
                               double *ess, int bf16) {
  int d = m->dx;
  double *lw = (double *)malloc(sizeof(double) * (size_t)N);
  double *dlw = (double *)malloc(sizeof(double) * (size_t)N);
  double *C = (double *)malloc(sizeof(double) * (size_t)N);
  double *U = (double *)malloc(sizeof(double) * (size_t)N);
  int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *Xo = (double *)malloc(sizeof(double) * (size_t)N * d);
  double mx, W, s2;

  or_propagate_learned(m, p, seed, filter, N, t, X, y, dlw, bf16);
  or_weights(m, N, X, y, lw);
  for (int i = 0; i < N; ++i) {
    lw[i] += dlw[i];
    if (isnan(lw[i])) lw[i] = -INFINITY;
  }
  int deg = or_normalise(N, lw, &mx, &W, &s2);
  if (logZ) {
    const double two_pi = 6.283185307179586476925286766559;
    if (deg)
      *logZ = -INFINITY;
    else
      *logZ += mx + log(W / (double)N) - 0.5 * m->dy * log(two_pi * m->obs_var);
  }
  if (ess) *ess = W * W / s2;
  if (mean_w) or_weighted_mean(N, d, X, lw, mx, mean_w);
  or_cdf(N, lw, mx, deg, C);
  or_sorted_uniforms(seed, filter, t, N, U);
  or_ancestors(N, C, U, A);
  or_gather(N, d, X, A, Xo);
  memcpy(X, Xo, sizeof(double) * (size_t)N * d);
  if (mean_post) or_mean(N, d, X, mean_post);
  if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)N);
  if (A_out) memcpy(A_out, A, sizeof(int32_t) * (size_t)N);
  free(lw); free(dlw); free(C); free(U); free(A); free(Xo);
  return deg;
}

void or_run_ensemble_learned(const or_model *m, const double *p, uint64_t seed,
                             int M, int N, int T, const double *y, double *est,
                             double *est_w, double *logZ, double *ess, int bf16) {
  int d = m->dx;
  double *X = (double *)malloc(sizeof(double) * (size_t)N * d);
  double *mp = (double *)malloc(sizeof(double) * (size_t)d);
  double *mw = (double *)malloc(sizeof(double) * (size_t)d);
  if (est) memset(est, 0, sizeof(double) * (size_t)T * d);
  if (est_w) memset(est_w, 0, sizeof(double) * (size_t)T * d);
  if (ess) memset(ess, 0, sizeof(double) * (size_t)T);
  for (int f = 0; f < M; ++f) {
    double lz = 0.0;
    or_init(m, seed, (uint32_t)f, N, X);
    for (int t = 1; t <= T; ++t) {
      double e;
      or_filter_interval_learned(m, p, seed, (uint32_t)f, N, t, X,
                                 y + (size_t)(t - 1) * m->dy, &lz, NULL, NULL, mp,
                                 mw, &e, bf16);
      for (int c = 0; c < d; ++c) {
        if (est) est[(size_t)(t - 1) * d + c] += mp[c] / (double)M;
        if (est_w) est_w[(size_t)(t - 1) * d + c] += mw[c] / (double)M;
      }
      if (ess) ess[t - 1] += e / (double)M;
    }
    if (logZ) logZ[f] = lz;
  }
  free(X); free(mp); free(mw);
}

/* Discrete OU x_{k+1} = phi x_k + sd sqrt(h) z_k, phi = 1 - theta h, observed
   as y = x_S + N(0, obs_var).  Given x_k = x, y - phi^{S-k} x is Gaussian with
   variance q_{S-k} + obs_var and covariance phi^{S-k-1} sd sqrt(h) with z_k,
   so (sd/sqrt(h)) E[z_k | x, y] is the expression below. */
double or_ou_optimal_u(const or_model *m, double x, double y, int k) {
  double phi = 1.0 - m->p[0] * m->h, sd = m->sd[0];
  int r = m->S - k;
  double a_r = pow(phi, r), a_r1 = pow(phi, r - 1), q = 0.0;
  for (int i = 0; i < r; ++i) q += sd * sd * m->h * pow(phi, 2 * i);
  return sd * sd * a_r1 * (y - a_r * x) / (q + m->obs_var);
}

/* ------------------------------------------------------------------------ */
/* Training data of the learned proposal (definitions in pf_oracle.h): model
   paths from the step noise and Euler-Maruyama steps above, with their own
   counters. */

static void train_prior(const or_model *m, const uint32_t key[2], uint32_t q, double *x) {
  uint32_t ctr[4];
  double z[4];
  for (int s = 0; s < m->dx; s += 4) {
    make_ctr(ctr, q, OR_TRAIN_RUN, 0xFFFFFFFFu, OR_P_TRAIN, (uint32_t)(s / 4));
    or_normals4(ctr, key, z);
    for (int l = 0; l < 4 && s + l < m->dx; ++l)
      x[s + l] = m->prior_mean[s + l] + m->prior_sd[s + l] * z[l];
  }
}

void or_train_run(const or_model *m, uint64_t seed, uint32_t q, int run_len, double *starts) {
  uint32_t key[2];
  or_key(seed, key);
  int d = m->dx;
  double *x = (double *)malloc(sizeof(double) * (size_t)d);
  double *z = (double *)malloc(sizeof(double) * (size_t)d);
  double *xn = (double *)malloc(sizeof(double) * (size_t)d);
  train_prior(m, key, q, x);
  for (int j = 0; j < run_len; ++j) {
    for (int s = 0; s < m->S; ++s) {
      uint32_t n = (uint32_t)(j * m->S + s);
      or_step_noise(m, key, OR_P_TRAIN, q, OR_TRAIN_RUN, n, z);
      or_em_step(m, x, z, xn);
      memcpy(x, xn, sizeof(double) * (size_t)d);
    }
    memcpy(starts + (size_t)j * d, x, sizeof(double) * (size_t)d);
  }
  free(x); free(z); free(xn);
}

void or_train_trajectory(const or_model *m, uint64_t seed, uint32_t r, const double *x0,
                         double *traj, double *y, double *zs) {
  uint32_t key[2], ctr[4];
  double q4[4];
  or_key(seed, key);
  int d = m->dx;
  double *x = (double *)malloc(sizeof(double) * (size_t)d);
  double *z = (double *)malloc(sizeof(double) * (size_t)d);
  double *xn = (double *)malloc(sizeof(double) * (size_t)d);
  memcpy(x, x0, sizeof(double) * (size_t)d);
  for (int k = 0; k < m->S; ++k) {
    memcpy(traj + (size_t)k * d, x, sizeof(double) * (size_t)d);
    or_step_noise(m, key, OR_P_TRAIN, r, OR_TRAIN_TRAJ, (uint32_t)k, z);
    if (zs) memcpy(zs + (size_t)k * d, z, sizeof(double) * (size_t)d);
    or_em_step(m, x, z, xn);
    memcpy(x, xn, sizeof(double) * (size_t)d);
  }
  double sy = sqrt(m->obs_var);
  for (int o = 0; o < m->dy; o += 4) {
    make_ctr(ctr, r, OR_TRAIN_TRAJ, 0xFFFFFFFFu, OR_P_TRAIN, (uint32_t)(o / 4));
    or_normals4(ctr, key, q4);
    for (int l = 0; l < 4 && o + l < m->dy; ++l) y[o + l] = x[m->obs_idx[o + l]] + sy * q4[l];
  }
  free(x); free(z); free(xn);
}

void or_train_tile(const or_model *m, uint64_t seed, int n_traj, int step, uint32_t b,
                   int *r, int *k, int *node0) {
  uint32_t key[2], ctr[4], w[4];
  or_key(seed, key);
  make_ctr(ctr, b, OR_TRAIN_BATCH, (uint32_t)step, OR_P_TRAIN, 0u);
  or_philox4x32_10(ctr, key, w);
  int tiles = m->J * m->J / 16;
  *r = (int)(((uint64_t)w[0] * (uint64_t)n_traj) >> 32);
  *k = (int)(w[1] % (uint32_t)m->S);
  *node0 = 16 * (int)(((uint64_t)w[2] * (uint64_t)tiles) >> 32);
}

void or_adam_step(int n, double *p, const double *g, double *mo, double *ve, double lr,
                  double beta1, double beta2, double eps, int t) {
  double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
  for (int i = 0; i < n; ++i) {
    mo[i] = beta1 * mo[i] + (1.0 - beta1) * g[i];
    ve[i] = beta2 * ve[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = mo[i] / c1, vh = ve[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
