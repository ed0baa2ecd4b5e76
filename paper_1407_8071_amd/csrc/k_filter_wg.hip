// k_filter_wg.hip -- the whole interval of a filter inside one workgroup
// (vector models, N up to 8192).
//
// One workgroup owns one filter for the interval, so no memory ever crosses
// workgroups and no grid-wide synchronisation or device-scope fence is
// needed (on MI355X a grid barrier across ~1300 workgroups measured ~60 us,
// more than the resampling work itself).  Per workgroup:
//   1. propagation: particle i = p * BD + tid (p = 0 .. ceil(N/BD)-1), read
//      through the previous interval's ancestor (fused gather), S Euler-
//      Maruyama steps in registers, log-weight to LDS and HBM, xbar to HBM;
//   2. normalisation: block maximum, w = exp(lw - mx) in FP64, the CDF by
//      chunked block scans into LDS (FP64), sum w^2, and sum w xbar;
//   3. sorted uniforms: thread t owns the contiguous k-range
//      [t*KPT, (t+1)*KPT); its exponentials E_j, their block exclusive scan
//      and the running sum give S_k, U_k = S_k / S_N;
//   4. ancestor search in the LDS CDF (bisection for the first k of the
//      thread, exponential search onward), ancestors to HBM, and the sum of
//      the resampled particles xbar^(a_k) read back from HBM (written by this
//      workgroup, so a workgroup barrier makes them visible);
//   5. the filter's estimates and log G update, written by thread 0.
// The cross-filter average is a separate small kernel.
#include "pf_internal.h"

namespace pfk {
namespace {

template <int D>
__device__ __forceinline__ void wg_drift(const ModelDev &md, const float x[D], float f[D]) {
  if constexpr (D == 3) {
    f[0] = md.p0 * (x[1] - x[0]);
    f[1] = md.p1 * x[0] - x[1] - x[0] * x[2];
    f[2] = x[0] * x[1] - md.p2 * x[2];
  } else {
    f[0] = -md.p0 * x[0];
  }
}

// S Euler-Maruyama steps with the FP32 increments summed in an offset from
// the start state (the same arithmetic as the batched propagation kernel).
template <int D>
__device__ __forceinline__ void wg_em(const ModelDev &md, Key key, uint32_t c0, uint32_t c1,
                                      int n0, float x[D]) {
  const int n1 = n0 + md.S;
  float x0[D], off[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x0[c] = x[c];
    off[c] = 0.f;
  }
  for (int q = n0 >> 2; (q << 2) < n1; ++q) {
    float z[4 * D];
#pragma unroll
    for (int j = 0; j < D; ++j)
      normals4(philox<2, 3>(c0, c1, (uint32_t)q, (P_PROP << 24) | (uint32_t)j, key), &z[4 * j]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 4 * q + r;
      if (n < n0 || n >= n1) continue;
      float xc[D], f[D];
#pragma unroll
      for (int c = 0; c < D; ++c) xc[c] = x0[c] + off[c];
      wg_drift<D>(md, xc, f);
#pragma unroll
      for (int c = 0; c < D; ++c) off[c] += fmaf(md.h, f[c], md.sq0 * z[r * D + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = x0[c] + off[c];
}

template <int D>
__device__ __forceinline__ float wg_loglik(const ModelDev &md, const float x[D], const float *y) {
  float acc = 0.f;
  for (int k = 0; k < md.dy; ++k) {
    const int o = gptr(md.obs_idx)[k];
    float xo = x[0];
#pragma unroll
    for (int c = 1; c < D; ++c)
      if (o == c) xo = x[c];
    const float r = gptr(y)[k] - xo;
    acc = fmaf(r, r, acc);
  }
  const float lw = -acc * md.inv2var;
  return (lw == lw) ? lw : -INFINITY;
}

struct ExpoWG {
  Key key;
  uint32_t m, t;
  int cached = -1;
  uint4 r;
  __device__ __forceinline__ double operator()(int j) {
    if ((j >> 2) != cached) {
      cached = j >> 2;
      r = philox<2, 3>((uint32_t)cached, m, t, P_RESAMPLE << 24, key);
    }
    const int l = j & 3;
    const uint32_t w = l == 0 ? r.x : l == 1 ? r.y : l == 2 ? r.z : r.w;
    return -log(u01d(w));
  }
};

// smallest i in [0, N) with C[i] > v (clamped to N - 1) without a known
// lower bound: bisection over the last entries of 64-entry blocks, then
// within the block (12 dependent LDS reads for N = 4096 instead of ~22 for a
// doubling search from 0)
__device__ __forceinline__ int lds_search_blocked(const double *C, int N, double v) {
  int a = 0, b = (N - 1) >> 6;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (C[min(64 * mid + 63, N - 1)] > v)
      b = mid;
    else
      a = mid + 1;
  }
  int lo = 64 * a, hi = min(64 * a + 63, N - 1);  // C[lo - 1] <= v
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] > v)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// smallest i in [0, N) with C[i] > v (clamped to N - 1), starting from the
// known lower bound lo (C[lo - 1] <= v)
__device__ __forceinline__ int lds_search(const double *C, int N, int lo, double v) {
  if (lo >= N - 1) return N - 1;
  if (C[lo] > v) return lo;
  int step = 1, known = lo, hi;
  while (true) {
    hi = known + step;
    if (hi >= N - 1) {
      hi = N - 1;
      break;
    }
    if (C[hi] > v) break;
    known = hi;
    step <<= 1;
  }
  int a = known + 1, b = hi;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (C[mid] > v)
      b = mid;
    else
      a = mid + 1;
  }
  return a;
}

template <int D, int BD>
__global__ void __launch_bounds__(BD)
k_filter_wg(const WgJob *__restrict__ jobs, const FusedEns *__restrict__ ens, IvArg iv,
            int parity, int pending, int resample_only) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  extern __shared__ double lds[];
  constexpr int NW = BD / 64;
  double *shd = lds;                       // NW doubles of reduction scratch
  float *shf = (float *)(lds + NW);        // NW floats
  double *C = lds + 2 * NW;                // [N] FP64 CDF
  const WgJob job = jobs[blockIdx.x];
  const FusedEns &E = ens[job.ens];
  const int m = job.filter, N = E.N, tid = threadIdx.x;
  float *lws = (float *)(C + N);           // [N] log-weights
  // (pointers from the ensemble table: global-address-space accesses)
  const gmem<float> *Xin = gptr(parity ? E.X1 : E.X0);
  gmem<float> *Xb = gptr(parity ? E.X0 : E.X1);  // xbar of this interval
  const size_t xo = (size_t)m * D * N;
  gmem<float> *lwg = gptr(E.lw + (size_t)m * N);

  // 1. propagation and weighting
  float lmax = -INFINITY;
  for (int i = tid; i < N; i += BD) {
    float lw;
    if (resample_only) {
      lw = lwg[i];
      lw = (lw == lw) ? lw : -INFINITY;
    } else {
      const int src = pending ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
      float x[D];
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] = Xin[xo + (size_t)c * N + src];
      wg_em<D>(E.md, E.key, (uint32_t)i, (uint32_t)m, (t - 1) * E.md.S, x);
#pragma unroll
      for (int c = 0; c < D; ++c) Xb[xo + (size_t)c * N + i] = x[c];
      lw = wg_loglik<D>(E.md, x, y + E.yoff);
      lwg[i] = lw;
    }
    lws[i] = lw;
    lmax = fmaxf(lmax, lw);
  }
  // 2. normalisation and the CDF in LDS
  const float mxf = block_max(lmax, shf);
  const bool deg = !(mxf > -INFINITY);
  const double mx = (double)mxf;
  double carry = 0.0, s2 = 0.0, sw[D];
#pragma unroll
  for (int c = 0; c < D; ++c) sw[c] = 0.0;
  for (int base = 0; base < N; base += BD) {
    const int i = base + tid;
    double w = 0.0;
    if (i < N) {
      w = deg ? 1.0 : exp((double)lws[i] - mx);
      s2 += w * w;
#pragma unroll
      for (int c = 0; c < D; ++c) sw[c] += w * (double)Xb[xo + (size_t)c * N + i];
    }
    double tot;
    const double ex = block_exscan(w, shd, &tot);
    if (i < N) C[i] = carry + (ex + w);
    carry += tot;
  }
  __syncthreads();
  const double W = C[N - 1];
  const double w2 = block_sum(s2, shd);
  double wsum[D];
#pragma unroll
  for (int c = 0; c < D; ++c) wsum[c] = block_sum(sw[c], shd);

  // 3. sorted uniforms from exponential spacings
  const int KPT = (N + BD - 1) / BD;
  const int k0 = tid * KPT, k1 = min(N, k0 + KPT);
  ExpoWG ex{E.key, (uint32_t)m, (uint32_t)t};
  double es = 0.0;
  for (int j = k0; j < k1; ++j) es += ex(j);
  double SN;
  const double eoff = block_exscan(es, shd, &SN);
  if (tid == 0) {
    ExpoWG tail{E.key, (uint32_t)m, (uint32_t)t};
    lds[2 * NW - 1] = tail(N);  // E_N, in the free slot after the float scratch
  }
  __syncthreads();
  SN += lds[2 * NW - 1];

  // 4. ancestors and the resampled sum
  double run = eoff, px[D];
#pragma unroll
  for (int c = 0; c < D; ++c) px[c] = 0.0;
  int i = 0;
  for (int k = k0; k < k1; ++k) {
    run += ex(k);
    const double v = (run / SN) * W;
    i = lds_search(C, N, (k == k0) ? 0 : i, v);
    gptr(E.A)[(size_t)m * N + k] = i;
#pragma unroll
    for (int c = 0; c < D; ++c) px[c] += (double)Xb[xo + (size_t)c * N + i];
  }
  double psum[D];
#pragma unroll
  for (int c = 0; c < D; ++c) psum[c] = block_sum(px[c], shd);

  // 5. the filter's estimates and log G_t^N
  if (tid == 0) {
    gmem<double> *f = gptr(E.fstat + (size_t)m * FREC);
    f[0] = mx;
    f[1] = W;
    f[2] = w2;
    f[3] = deg ? 1.0 : 0.0;
    f[4] = SN;
    f[5] = deg ? -INFINITY : f[5] + mx + log(W / (double)N) + E.lognorm;
    f[6] = W * W / w2;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      gptr(E.fmean)[(size_t)m * D + c] = psum[c] / (double)N;
      gptr(E.fmeanw)[(size_t)m * D + c] = wsum[c] / W;
    }
  }
}

// Resampling of one filter per workgroup from its log-weights: normalisation,
// the LDS CDF, the sorted uniforms, the ancestors, their offspring counts n_i
// and log G.  Thread t owns the contiguous elements [t*P, (t+1)*P) (P =
// ceil(N/BD) <= RS_MAX_P, and 1 below 1024 threads) for every quantity: its log-weights, weights and
// (vector models) xbar stay in registers; the CDF and the uniforms each take
// one sequential scan per thread, and their two block scans run as one.
// The exponential spacings do not depend on the weights and are drawn while
// the log-weights load.  Grid model (D = 0):
// the counts go to HBM for the state-wide estimator.  Vector models (D = 1,
// 3): the workgroup also forms the post-resampling estimate
// sum_i n_i xbar_i / N and the weighted estimate sum_i w_i xbar_i / W.
constexpr int RS_MAX_P = 8;

typedef float f4v __attribute__((ext_vector_type(4)));

// Elements k0 .. k0 + PM - 1 of a row of N floats into registers, indices
// clamped into the row.  vec4: k0 and N are multiples of 4 and the row
// starts on a 16-byte boundary, so 4-element chunks are either inside the
// row or wholly past its end (then the last chunk is read instead).
template <int PM>
__device__ __forceinline__ void load_span(const gmem<float> *row, int k0, int N, bool vec4,
                                          float out[PM]) {
  if constexpr (PM % 4 == 0) {
    if (vec4) {
#pragma unroll
      for (int j = 0; j < PM / 4; ++j) {
        const f4v v = *(const gmem<f4v> *)(row + min(k0 + 4 * j, N - 4));
#pragma unroll
        for (int q = 0; q < 4; ++q) out[4 * j + q] = v[q];
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < PM; ++e) out[e] = row[min(k0 + e, N - 1)];
}

// PM: elements per thread the registers hold, at least ceil(N / BD) for every
// filter of the launch (1 below 1024 threads, which serve filters of N <= BD).
// CUSTOM: the launch serves ensembles with another scheme or the ESS schedule
// (compiled apart, so that the multinomial body keeps its registers).
template <int BD, int D, int PM, bool CUSTOM>
__device__ __forceinline__ void resample_wg(const WgJob *__restrict__ jobs,
                                            const FusedEns *__restrict__ ens, IvArg iv,
                                            int32_t *const *__restrict__ counts, int xb_parity,
                                            int stage) {
  const int t = iv_t(iv);
  extern __shared__ double lds[];
  constexpr int NW = BD / 64;
  constexpr int DD = D > 0 ? D : 1;
  double *shd = lds;                 // 8 * NW doubles: multi-value reductions
  float *shf = (float *)(lds + 8 * NW);
  double *C = lds + 9 * NW;          // [N] CDF
  const WgJob job = jobs[blockIdx.x];
  const FusedEns &E = ens[job.ens];
  const int m = job.filter, N = E.N, tid = threadIdx.x;
  int *cnt = (int *)(C + N);         // [N] offspring counts
  const int P = (N + BD - 1) / BD;
  const int k0 = min(N, tid * P), k1 = min(N, k0 + P);
  // (pointers from the ensemble table: global-address-space accesses)
  const gmem<float> *lwg = gptr(E.lw + (size_t)m * N);
  constexpr int NR = 1 + 2 * DD;         // sums of the final reduction
  constexpr int T5 = BD > 64 ? 64 : NR;  // the thread that updates log G
  // that thread reads the running evidence now, so that its latency is hidden
  const double lg_prev = tid == T5 ? gptr(E.fstat)[(size_t)m * FREC + 5] : 0.0;
  const gmem<float> *Xb = gptr((xb_parity ? E.X1 : E.X0) + (size_t)m * DD * N);
  // 1. this thread's log-weights.  The loads are unconditional (index
  // clamped; a slot past the thread's range gets weight 0 and count 0), so
  // that they all issue at once; they are first used after step 2.  Where
  // every thread's range starts on a 16-byte boundary (P and N multiples of
  // 4) they are 16-byte loads: one instruction per 4 elements instead of 4
  // lane-strided ones that each touch 4 times the cache lines they use.
  const bool vec4 = PM % 4 == 0 && P % 4 == 0 && N % 4 == 0;
  // the ensemble's scheme and schedule (uniform over the workgroup)
  const int scheme = CUSTOM ? E.scheme : RS_MULTINOMIAL;
  // ESS schedule: the carried log-weights join the interval's ones here.
  // Auxiliary filters: stage 1 resamples from the pilot weights (which carry
  // them already), stage 0 normalises the second-stage weights and carries
  // them (never resamples)
  const bool sched = CUSTOM && E.ess_thr > 0.0;
  const bool apf = CUSTOM && E.apf != 0;
  float lw[PM], lc[PM];
  load_span<PM>(lwg, k0, N, vec4, lw);
  if (sched) load_span<PM>(gptr(E.lwc + (size_t)m * N), k0, N, vec4, lc);
#pragma unroll
  for (int e = 0; e < PM; ++e)
    if (k0 + e < k1) cnt[k0 + e] = 0;
  // 2. exponential spacings over the same elements (they do not depend on
  // the weights: computed while the loads are in flight); multinomial and
  // residual resampling draw from them
  ExpoWG ex{E.key, (uint32_t)m, (uint32_t)t};
  double eg[PM], es = 0.0;
  const bool spacings = scheme == RS_MULTINOMIAL || scheme == RS_RESIDUAL;
#pragma unroll
  for (int e = 0; e < PM; ++e) {
    eg[e] = (spacings && k0 + e < k1) ? ex(k0 + e) : 0.0;
    es += eg[e];
  }
  // the last thread, whose range is last (or empty), adds E_N: it enters
  // the total S_N but no thread's exclusive prefix
  if (spacings && tid == BD - 1) {
    ExpoWG tail{E.key, (uint32_t)m, (uint32_t)t};
    es += tail(N);
  }
  // 3. the filter maximum, the weights and their thread-local inclusive
  // scan; one block scan of the weights and the spacings -> CDF, S_N.  With
  // the ESS schedule a particle's log-weight is its carried log-weight plus
  // the interval's log-likelihood, and the sum replaces the stored value
  float lmax = -INFINITY;
#pragma unroll
  for (int e = 0; e < PM; ++e) {
    lw[e] = (k0 + e < k1 && lw[e] == lw[e]) ? lw[e] : -INFINITY;
    if (sched) {
      lw[e] += lc[e];
      lw[e] = lw[e] == lw[e] ? lw[e] : -INFINITY;
      if (k0 + e < k1) gptr(E.lw)[(size_t)m * N + k0 + e] = lw[e];
    }
    lmax = fmaxf(lmax, lw[e]);
  }
  const float mxf = block_max(lmax, shf);
  const bool deg = !(mxf > -INFINITY);
  const double mx = (double)mxf;
  // xbar (vector models), first used in step 5: issued only now, so that
  // the log-weights of every workgroup did not share the memory system with
  // three times their volume, and arriving under steps 3-4
  float xb[DD][PM];
  if constexpr (D > 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) load_span<PM>(Xb + (size_t)c * N, k0, N, vec4, xb[c]);
  }
  double w[PM], run = 0.0, s2 = 0.0;
#pragma unroll
  for (int e = 0; e < PM; ++e) {
    w[e] = 0.0;
    if (k0 + e < k1) w[e] = deg ? 1.0 : exp((double)lw[e] - mx);
    run += w[e];
    s2 += w[e] * w[e];
  }
  double sc[2], tot[2];
  block_exscan2(run, es, shd, sc, tot);
  {
    double c = sc[0];
#pragma unroll
    for (int e = 0; e < PM; ++e) {
      c += w[e];
      if (k0 + e < k1) C[k0 + e] = c;
    }
  }
  const double eoff = sc[1], SN = tot[1];
  __syncthreads();  // publishes C
  const double W = C[N - 1];
  // the schedule's decision: resample every interval, or only when the ESS
  // (sum w)^2 / sum w^2 falls below ess_thr N (and always when degenerate)
  bool resample = true;
  if (sched) {
    const double w2 = block_sum(s2, shd);
    resample = deg || W * W / w2 < E.ess_thr * (double)N;
  }
  if (apf) resample = stage == 1;
  gmem<int32_t> *Ag = gptr(E.A + (size_t)m * N);
  if (!resample) {
    // 4'. the particles stay (identity ancestors, one offspring each) and
    // carry their log-weights, normalised to mean weight 1
    const double shift = mx + log(W / (double)N);
#pragma unroll
    for (int e = 0; e < PM; ++e) {
      const int k = k0 + e;
      if (k < k1) {
        Ag[k] = k;
        cnt[k] = 1;
        gptr(E.lwc)[(size_t)m * N + k] = deg ? 0.f : (float)((double)lw[e] - shift);
      }
    }
  } else {
    if (sched) {
#pragma unroll
      for (int e = 0; e < PM; ++e)
        if (k0 + e < k1) gptr(E.lwc)[(size_t)m * N + k0 + e] = 0.f;
    }
    if (scheme == RS_RESIDUAL) {
      // 4r. residual resampling: floor(N w_i / W) copies of particle i, then
      // R = N - sum of the floors multinomial draws from the fractional
      // parts (sorted uniforms from the spacings of E_0 .. E_R), the
      // ancestors listed in index order
      double nsum = 0.0, rsum = 0.0;
#pragma unroll
      for (int e = 0; e < PM; ++e)
        if (k0 + e < k1) {
          const double nw = (double)N * w[e] / W;
          const double fl = floor(nw);
          nsum += fl;
          rsum += nw - fl;
        }
      double sc2[2], tot2[2];
      block_exscan2(nsum, rsum, shd, sc2, tot2);  // (its first barrier: C[N-1] was read)
      const int R = N - (int)tot2[0];
      {
        double c = sc2[1];
#pragma unroll
        for (int e = 0; e < PM; ++e)
          if (k0 + e < k1) {
            const double nw = (double)N * w[e] / W;
            c += nw - floor(nw);
            C[k0 + e] = c;  // the residual CDF replaces the CDF
          }
      }
      // S_R, the spacings' prefix at R, from the thread that owns index R
      double *sR = (double *)(((uintptr_t)(cnt + N) + 7) & ~(uintptr_t)7);
      if (R < N) {
        if (k0 <= R && R < k1) {
          double a = eoff;
#pragma unroll
          for (int e = 0; e < PM; ++e)
            if (k0 + e <= R) a += eg[e];
          *sR = a;
        }
      } else if (tid == 0) {
        *sR = SN;
      }
      __syncthreads();
      const double SR = *sR, Wr = C[N - 1];
      double sacc = eoff;
      int i = 0;
#pragma unroll
      for (int e = 0; e < PM; ++e) {
        const int k = k0 + e;
        if (k < k1 && k < R) {
          sacc += eg[e];
          const double v = (sacc / SR) * Wr;
          i = e == 0 ? lds_search_blocked(C, N, v) : lds_search(C, N, i, v);
          atomicAdd(cnt + i, 1);
        }
      }
      __syncthreads();
      // total offspring of each particle; positions from one block scan
      int o[PM];
      double osum = 0.0;
#pragma unroll
      for (int e = 0; e < PM; ++e) {
        o[e] = 0;
        if (k0 + e < k1) o[e] = (int)floor((double)N * w[e] / W) + cnt[k0 + e];
        osum += (double)o[e];
      }
      double otot;
      int pos = (int)block_exscan(osum, shd, &otot);
#pragma unroll
      for (int e = 0; e < PM; ++e) {
        const int k = k0 + e;
        if (k < k1) {
          for (int j = 0; j < o[e]; ++j) Ag[pos++] = k;
          cnt[k] = o[e];
        }
      }
    } else {
      // 4. ancestors in the LDS CDF and the offspring counts: the sorted
      // points are exponential spacings (multinomial), one uniform offset on
      // the lattice k / N (systematic) or one uniform in each stratum
      // [k / N, (k + 1) / N) (stratified)
      double sacc = eoff;
      int i = 0;
      const double usys =
          scheme == RS_SYSTEMATIC
              ? u01d(philox(0u, (uint32_t)m, (uint32_t)t, (P_RESAMPLE << 24) | 1u, E.key).x)
              : 0.0;
      int cached = -1;
      uint4 rq = make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < PM; ++e) {
        const int k = k0 + e;
        if (k < k1) {
          double v;
          if (scheme == RS_MULTINOMIAL) {
            sacc += eg[e];
            v = (sacc / SN) * W;
          } else if (scheme == RS_SYSTEMATIC) {
            v = (((double)k + usys) / (double)N) * W;
          } else {
            if ((k >> 2) != cached) {
              cached = k >> 2;
              rq = philox((uint32_t)cached, (uint32_t)m, (uint32_t)t, (P_RESAMPLE << 24) | 2u,
                          E.key);
            }
            const int l = k & 3;
            const uint32_t wq = l == 0 ? rq.x : l == 1 ? rq.y : l == 2 ? rq.z : rq.w;
            v = (((double)k + u01d(wq)) / (double)N) * W;
          }
          i = e == 0 ? lds_search_blocked(C, N, v) : lds_search(C, N, i, v);
          Ag[k] = i;
          atomicAdd(cnt + i, 1);
        }
      }
    }
  }
  __syncthreads();
  // 5. post-resampling sums, one fused block reduction, outputs
  double red[1 + 2 * DD];
  red[0] = s2;
  if constexpr (D > 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double px = 0.0, wx = 0.0;
#pragma unroll
      for (int e = 0; e < PM; ++e) {
        if (k0 + e < k1) px += (double)cnt[k0 + e] * (double)xb[c][e];
        wx += w[e] * (double)xb[c][e];
      }
      red[1 + c] = resample ? px : wx;  // kept particles: the weighted estimate
      red[1 + D + c] = wx;
    }
  } else {
    gmem<int32_t> *cg = gptr(counts[job.ens] + (size_t)m * N);
    for (int j = tid; j < N; j += BD) cg[j] = cnt[j];
    red[1] = red[2] = 0.0;
  }
  // thread r < NR folds sum r; the quotients of the outputs are taken side
  // by side in those lanes (one division sequence, per-lane operands), and
  // the logarithm of log G by thread T5 (another wave, where there is one)
  const double a = block_sum_multi_lane<NR>(red, shd);
  gmem<double> *f = gptr(E.fstat + (size_t)m * FREC);
  if (tid < (D > 0 ? NR : 1)) {
    double num = a, den = W;
    gmem<double> *dst = f + 6;
    if (tid == 0) {
      num = W * W;  // ESS = W^2 / sum w^2
      den = a;
    } else if (tid <= D) {
      den = resample ? (double)N : W;
      dst = gptr(E.fmean + (size_t)m * D + (tid - 1));
    } else {
      dst = gptr(E.fmeanw + (size_t)m * D + (tid - 1 - D));
    }
    *dst = num / den;
    if (tid == 0) {
      f[0] = mx;
      f[1] = W;
      f[2] = a;  // sum w^2
      f[3] = deg ? 1.0 : 0.0;
      f[4] = SN;
      f[FREC_KEPT] = resample ? 0.0 : 1.0;
    }
  }
  // (the first stage of an auxiliary filter adds its factor of the
  // evidence without the Gaussian constant, which the second stage adds)
  if (tid == T5)
    f[5] = deg ? -INFINITY
               : lg_prev + mx + log(W / (double)N) + (stage == 1 ? 0.0 : E.lognorm);
}

// The kernel: PMAX is the largest ceil(N / BD) of the launch's filters; each
// workgroup runs the body compiled for its own filter's count (a uniform
// branch), so that small filters in a launch with large ones read no more
// than they need.
template <int BD, int D, int PMAX, bool CUSTOM>
__global__ void __launch_bounds__(BD)
k_resample_wg(const WgJob *__restrict__ jobs, const FusedEns *__restrict__ ens, IvArg iv,
              int32_t *const *__restrict__ counts, int xb_parity, int stage) {
  if constexpr (PMAX == 1) {
    resample_wg<BD, D, 1, CUSTOM>(jobs, ens, iv, counts, xb_parity, stage);
  } else {
    const int P = (ens[jobs[blockIdx.x].ens].N + BD - 1) / BD;
    if (P <= 1)
      resample_wg<BD, D, 1, CUSTOM>(jobs, ens, iv, counts, xb_parity, stage);
    else if (P <= 2 || PMAX == 2)
      resample_wg<BD, D, (PMAX >= 2 ? 2 : 1), CUSTOM>(jobs, ens, iv, counts, xb_parity, stage);
    else if (P <= 4 || PMAX == 4)
      resample_wg<BD, D, (PMAX >= 4 ? 4 : 1), CUSTOM>(jobs, ens, iv, counts, xb_parity, stage);
    else
      resample_wg<BD, D, PMAX, CUSTOM>(jobs, ens, iv, counts, xb_parity, stage);
  }
}

// Offspring counts n_i = #{k : a_k = i} of every filter from its ancestors.
__global__ void __launch_bounds__(256)
k_offspring_counts(int N, const int32_t *__restrict__ A, int32_t *__restrict__ cnt) {
  const int m = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  atomicAdd(cnt + (size_t)m * N + min(max(A[(size_t)m * N + k], 0), N - 1), 1);
}

}  // namespace

// LDS bytes of a resampling workgroup (BD threads) for filters of up to N
// particles: reduction scratch, the CDF, the offspring counts.
size_t resample_wg_lds(int N, int BD) {
  return sizeof(double) * (9 * (size_t)(BD / 64) + 2) + sizeof(double) * (size_t)N +
         sizeof(int) * (size_t)N;
}

hipError_t launch_resample_wg(int D, int BD, const WgJob *d_jobs, int n_jobs, int max_n,
                              const FusedEns *d_ens, IvArg iv, int32_t *const *d_counts,
                              int xb_parity, bool custom, int stage, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  const size_t lds = resample_wg_lds(max_n, BD);
  const int pm = BD < 1024 ? 1 : (max_n <= 1024 ? 1 : max_n <= 2048 ? 2 : max_n <= 4096 ? 4 : 8);
  if (BD < 1024 && max_n > BD) return hipErrorInvalidValue;
  if (max_n > RS_MAX_P * 1024) return hipErrorInvalidValue;
#define PF_RS_LAUNCH(B, DD, P)                                                                  \
  do {                                                                                          \
    if (custom)                                                                                 \
      k_resample_wg<B, DD, P, true><<<n_jobs, B, lds, s>>>(d_jobs, d_ens, iv, d_counts, xb_parity, stage);  \
    else                                                                                        \
      k_resample_wg<B, DD, P, false><<<n_jobs, B, lds, s>>>(d_jobs, d_ens, iv, d_counts, xb_parity, stage); \
  } while (0)
#define PF_RS_BD(DD)                 \
  if (BD == 64) PF_RS_LAUNCH(64, DD, 1); \
  else if (BD == 128) PF_RS_LAUNCH(128, DD, 1); \
  else if (BD == 256) PF_RS_LAUNCH(256, DD, 1); \
  else if (BD == 512) PF_RS_LAUNCH(512, DD, 1); \
  else if (pm == 1) PF_RS_LAUNCH(1024, DD, 1); \
  else if (pm == 2) PF_RS_LAUNCH(1024, DD, 2); \
  else if (pm == 4) PF_RS_LAUNCH(1024, DD, 4); \
  else PF_RS_LAUNCH(1024, DD, 8)
  if (D == 0) {
    PF_RS_BD(0);
  } else if (D == 1) {
    PF_RS_BD(1);
  } else {
    PF_RS_BD(3);
  }
#undef PF_RS_BD
#undef PF_RS_LAUNCH
  return hipGetLastError();
}

hipError_t launch_offspring_counts(const EnsDev &e, int32_t *cnt, hipStream_t s) {
  hipError_t err = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)e.M * e.N, s);
  if (err != hipSuccess) return err;
  dim3 g((unsigned)((e.N + 255) / 256), (unsigned)e.M);
  k_offspring_counts<<<g, 256, 0, s>>>(e.N, e.A, cnt);
  return hipGetLastError();
}

// LDS bytes of a workgroup that owns a filter of N particles.
size_t filter_wg_lds(int N, int BD) {
  return sizeof(double) * (2 * (size_t)(BD / 64) + 2) + sizeof(double) * (size_t)N +
         sizeof(float) * (size_t)N;
}

hipError_t launch_filter_wg(int D, int BD, const WgJob *d_jobs, int n_jobs, int max_n,
                            const FusedEns *d_ens, IvArg iv, int parity, int pending,
                            int resample_only, hipStream_t s) {
  const size_t lds = filter_wg_lds(max_n, BD);
#define PF_WG_LAUNCH(DD, B)                                                                  \
  k_filter_wg<DD, B><<<n_jobs, B, lds, s>>>(d_jobs, d_ens, iv, parity, pending, resample_only)
  if (D == 3) {
    if (BD == 256) PF_WG_LAUNCH(3, 256);
    else if (BD == 512) PF_WG_LAUNCH(3, 512);
    else PF_WG_LAUNCH(3, 1024);
  } else {
    if (BD == 256) PF_WG_LAUNCH(1, 256);
    else if (BD == 512) PF_WG_LAUNCH(1, 512);
    else PF_WG_LAUNCH(1, 1024);
  }
#undef PF_WG_LAUNCH
  return hipGetLastError();
}

hipError_t set_filter_wg_lds_limit() {
  // allow the largest dynamic LDS request of either kernel (N = 8192 at
  // BD = 1024)
  const size_t fw = filter_wg_lds(WG_MAX_N, 1024), rw = resample_wg_lds(WG_MAX_N, 1024);
  const int bytes = (int)(fw > rw ? fw : rw);
  hipError_t e;
  e = hipFuncSetAttribute((const void *)k_filter_wg<3, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_filter_wg<3, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_filter_wg<3, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_filter_wg<1, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_filter_wg<1, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
#define PF_RS_PAIR(B, DD, P) \
  (const void *)k_resample_wg<B, DD, P, false>, (const void *)k_resample_wg<B, DD, P, true>
  const void *rs[] = {PF_RS_PAIR(256, 0, 1),  PF_RS_PAIR(512, 0, 1),  PF_RS_PAIR(1024, 0, 1),
                      PF_RS_PAIR(1024, 0, 2), PF_RS_PAIR(1024, 0, 4), PF_RS_PAIR(1024, 0, 8),
                      PF_RS_PAIR(256, 1, 1),  PF_RS_PAIR(512, 1, 1),  PF_RS_PAIR(1024, 1, 1),
                      PF_RS_PAIR(1024, 1, 2), PF_RS_PAIR(1024, 1, 4), PF_RS_PAIR(1024, 1, 8),
                      PF_RS_PAIR(256, 3, 1),  PF_RS_PAIR(512, 3, 1),  PF_RS_PAIR(1024, 3, 1),
                      PF_RS_PAIR(1024, 3, 2), PF_RS_PAIR(1024, 3, 4), PF_RS_PAIR(1024, 3, 8)};
#undef PF_RS_PAIR
  for (const void *f : rs) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipFuncSetAttribute((const void *)k_filter_wg<1, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace pfk
