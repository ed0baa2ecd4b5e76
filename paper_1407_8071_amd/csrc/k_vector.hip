// k_vector.hip -- kernels of the low-dimensional vector models (1-D OU test
// model, stochastic Lorenz 63).  One thread per particle; the state lives in
// registers for all S Euler-Maruyama steps of an interval, and the Philox
// normals are generated in the register file four steps at a time.
// Particle layout: float32 [M][D][N] (structure of arrays per filter), so
// every component load and store is coalesced across a wavefront.
#include "pf_internal.h"

namespace pfk {
namespace {

constexpr int VEC_BLOCK = 256;

// Drift of the model (Lorenz 63: Sec. 4.1, eqs. (eqDiscreteLorenz-1..3)).
template <int D>
__device__ __forceinline__ void drift(const ModelDev &md, const float x[D], float f[D]) {
  if constexpr (D == 3) {
    f[0] = md.p0 * (x[1] - x[0]);
    f[1] = md.p1 * x[0] - x[1] - x[0] * x[2];
    f[2] = x[0] * x[1] - md.p2 * x[2];
  } else {
    f[0] = -md.p0 * x[0];
  }
}

// S Euler-Maruyama steps n = n0 .. n0+S-1 of one particle (c0 = particle,
// c1 = filter or stream id).  The normals of a quad of steps q = n/4 come
// from D Philox calls (sub-blocks 0..D-1): normal l = (n%4)*D + c of the
// quad feeds component c of step n.
// The increments h f(x) + sd sqrt(h) z (~1e-2) are summed in an FP32 offset
// from the interval's start state x0 (order 10): the drift sees
// fl(x0 + offset) and the state is rounded once at the end, so the rounding
// of S additions to a state of order 10 never accumulates (4 operations per
// component and step, against 6 for a compensated sum of the same accuracy).
template <int D>
__device__ __forceinline__ void em_steps(const ModelDev &md, Key key, uint32_t purpose,
                                         uint32_t c0, uint32_t c1, int n0, int S, float x[D]) {
  const int n1 = n0 + S;
  float x0[D], off[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x0[c] = x[c];
    off[c] = 0.f;
  }
  for (int q = n0 >> 2; (q << 2) < n1; ++q) {
    float z[4 * D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const uint4 w = philox<2, 3>(c0, c1, (uint32_t)q, (purpose << 24) | (uint32_t)j, key);
      normals4(w, &z[4 * j]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 4 * q + r;
      if (n < n0 || n >= n1) continue;
      float xc[D], f[D];
#pragma unroll
      for (int c = 0; c < D; ++c) xc[c] = x0[c] + off[c];
      drift<D>(md, xc, f);
#pragma unroll
      for (int c = 0; c < D; ++c) off[c] += fmaf(md.h, f[c], md.sq0 * z[r * D + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = x0[c] + off[c];
}

template <int D>
__device__ __forceinline__ float loglik(const ModelDev &md, const float x[D], const float *y) {
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

template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_init(ModelDev md, Key key, int N, float *__restrict__ X) {
  const int m = blockIdx.y;
  const int i = blockIdx.x * VEC_BLOCK + threadIdx.x;
  if (i >= N) return;
  float z[4];
  normals4(philox((uint32_t)i, (uint32_t)m, 0u, P_INIT << 24, key), z);
#pragma unroll
  for (int c = 0; c < D; ++c)
    X[((size_t)m * D + c) * N + i] = md.prior_mean[c] + md.prior_sd[c] * z[c];
}

// Algorithm 1 step 2(a): xbar^(i) ~ tau_t(.|x^(anc_i)); optionally also the
// log-weight (fused weighting) when lw != nullptr.
template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_propagate(ModelDev md, Key key, int N, int t, const float *__restrict__ Xin,
                const int32_t *__restrict__ anc, float *__restrict__ Xout,
                float *__restrict__ lw, const float *__restrict__ y) {
  const int m = blockIdx.y;
  const int i = blockIdx.x * VEC_BLOCK + threadIdx.x;
  if (i >= N) return;
  const int src = anc ? min(max(anc[(size_t)m * N + i], 0), N - 1) : i;
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = Xin[((size_t)m * D + c) * N + src];
  em_steps<D>(md, key, P_PROP, (uint32_t)i, (uint32_t)m, (t - 1) * md.S, md.S, x);
#pragma unroll
  for (int c = 0; c < D; ++c) Xout[((size_t)m * D + c) * N + i] = x[c];
  if (lw) lw[(size_t)m * N + i] = loglik<D>(md, x, y);
}

// Batched propagation and weighting for the fused path: tile g of the table
// is (ensemble, filter, first particle) and holds up to 256 particles; every
// particle is read through the previous ancestors when `pending`.  For a
// tiled ensemble the workgroup also raises the maximum key of the resampling
// tile that holds its particles (a propagation tile of 64..1024 never
// straddles one of 4096) with one atomic.
template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_prop_batched(const int4 *__restrict__ tiles, const FusedEns *__restrict__ ens, IvArg iv,
                   int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const int4 tl = tiles[blockIdx.x];
  const FusedEns &E = ens[tl.x];
  const int m = tl.y, i = tl.z + threadIdx.x, N = E.N;
  float l = -INFINITY;
  if (i < N) {
    // (pointers from the ensemble table: global-address-space accesses)
    const gmem<float> *Xin = gptr(parity ? E.X1 : E.X0);
    gmem<float> *Xout = gptr(parity ? E.X0 : E.X1);
    // (an auxiliary filter's particles always come through the ancestors its
    // first stage has just drawn)
    const bool thru = pending || E.apf;
    const int src = thru ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
    float x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = Xin[((size_t)m * D + c) * N + src];
    em_steps<D>(E.md, E.key, P_PROP, (uint32_t)i, (uint32_t)m, (t - 1) * E.md.S, E.md.S, x);
#pragma unroll
    for (int c = 0; c < D; ++c) Xout[((size_t)m * D + c) * N + i] = x[c];
    l = loglik<D>(E.md, x, y + E.yoff);
    // auxiliary filter: the second-stage weight divides by the pilot
    // likelihood of the particle's ancestor
    if (E.apf) l -= gptr(E.lpil)[(size_t)m * N + src];
    l = l == l ? l : -INFINITY;
    gptr(E.lw)[(size_t)m * N + i] = l;
  }
  if (E.mxkey) {  // (the same for the whole workgroup)
    // every lane takes part: lanes past N carry -inf
    __shared__ float wmax[VEC_BLOCK / 64];
    const float wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      float v = wmax[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmaxf(v, wmax[w]);
      if (v > -INFINITY)
        __hip_atomic_fetch_max(gptr(E.mxkey) + (size_t)m * E.T + tl.z / TILE, ord_key(v),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Auxiliary filters: the pilot of particle i -- its noise-free S-step Euler
// path mu_i, summed in the same FP32 offset form as the stochastic steps --
// and the first-stage log-weight lwc_i + log g(y | mu_i); the pilot
// log-likelihood is kept for the second stage.
template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_pilot(const FusedEns *__restrict__ ens, int e, IvArg iv, int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const FusedEns &E = ens[e];
  const int m = blockIdx.y, i = blockIdx.x * VEC_BLOCK + threadIdx.x, N = E.N;
  if (i >= N) return;
  const gmem<float> *Xin = gptr(parity ? E.X1 : E.X0);
  const int src = pending ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
  const ModelDev md = E.md;
  float x0[D], off[D], x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x0[c] = Xin[((size_t)m * D + c) * N + src];
    off[c] = 0.f;
  }
  for (int st = 0; st < md.S; ++st) {
    float f[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = x0[c] + off[c];
    drift<D>(md, x, f);
#pragma unroll
    for (int c = 0; c < D; ++c) off[c] = fmaf(md.h, f[c], off[c]);
  }
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = x0[c] + off[c];
  const float pl = loglik<D>(md, x, y + E.yoff);
  const size_t o = (size_t)m * N + i;
  gptr(E.lpil)[o] = pl;
  const float lam = pl + gptr(E.lwc)[o];
  gptr(E.lw)[o] = lam == lam ? lam : -INFINITY;
}

template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_loglik(ModelDev md, int N, const float *__restrict__ X, const float *__restrict__ y,
             float *__restrict__ lw) {
  const int m = blockIdx.y;
  const int i = blockIdx.x * VEC_BLOCK + threadIdx.x;
  if (i >= N) return;
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = X[((size_t)m * D + c) * N + i];
  lw[(size_t)m * N + i] = loglik<D>(md, x, y);
}

// Algorithm 1 step 2(b): x^(k) = xbar^(a_k).
template <int D>
__global__ void __launch_bounds__(VEC_BLOCK)
k_vec_gather(int N, const int32_t *__restrict__ A, const float *__restrict__ Xin,
             float *__restrict__ Xout) {
  const int m = blockIdx.y;
  const int k = blockIdx.x * VEC_BLOCK + threadIdx.x;
  if (k >= N) return;
  const int a = min(max(A[(size_t)m * N + k], 0), N - 1);
#pragma unroll
  for (int c = 0; c < D; ++c) Xout[((size_t)m * D + c) * N + k] = Xin[((size_t)m * D + c) * N + a];
}

// Per-tile partial sums of the post-resampling particles (for (f, pi_t^N))
// and of the weighted pre-resampling particles (for sum_i w^(i) xbar^(i)).
// 1024 threads per tile of 4096, 4 lane-strided elements each, whose loads
// (and the gathers through the ancestors) issue together; one reduction of
// all 2 D sums.
constexpr int EST_THREADS = 1024, EST_PER_THREAD = TILE / EST_THREADS;
template <int D>
__global__ void __launch_bounds__(EST_THREADS)
k_vec_estimate_tiles(int N, int T, const float *__restrict__ Xpost, const float *__restrict__ Xpre,
                     const int32_t *__restrict__ anc, const float *__restrict__ lw,
                     const double *__restrict__ fstat, double *__restrict__ mpart,
                     double *__restrict__ wpart) {
  __shared__ double sh[2 * D * (EST_THREADS / 64)];
  const int m = blockIdx.y, q = blockIdx.x;
  const double mx = fstat[(size_t)m * FREC + 0];
  const bool deg = fstat[(size_t)m * FREC + 3] != 0.0;
  double v[2 * D];
#pragma unroll
  for (int c = 0; c < 2 * D; ++c) v[c] = 0.0;
#pragma unroll
  for (int e = 0; e < EST_PER_THREAD; ++e) {
    const int i = q * TILE + e * EST_THREADS + threadIdx.x;
    if (i < N) {
      const double w = deg ? 1.0 : exp((double)lw[(size_t)m * N + i] - mx);
      // post-resampling particle k = i: stored, or xbar read through a_i
      const int src = anc ? min(max(anc[(size_t)m * N + i], 0), N - 1) : i;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        v[c] += (double)Xpost[((size_t)m * D + c) * N + src];
        v[D + c] += w * (double)Xpre[((size_t)m * D + c) * N + i];
      }
    }
  }
  block_sum_multi_t0<2 * D>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      mpart[((size_t)m * T + q) * D + c] = v[c];
      wpart[((size_t)m * T + q) * D + c] = v[D + c];
    }
  }
}

// Truth path on the dedicated truth stream (one thread) and its observations.
template <int D>
__global__ void k_vec_simulate(ModelDev md, Key key, int T, float obs_sd,
                               float *__restrict__ xtrue, float *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float x[D], z[4];
  normals4(philox(0u, TRUTH_STREAM, 0u, P_TRUTH_INIT << 24, key), z);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x[c] = md.prior_mean[c] + md.prior_sd[c] * z[c];
    xtrue[c] = x[c];
  }
  for (int t = 1; t <= T; ++t) {
    em_steps<D>(md, key, P_TRUTH_NOISE, 0u, TRUTH_STREAM, (t - 1) * md.S, md.S, x);
#pragma unroll
    for (int c = 0; c < D; ++c) xtrue[(size_t)t * D + c] = x[c];
    for (int k = 0; k < md.dy; k += 4) {
      normals4(philox(0u, TRUTH_STREAM, (uint32_t)t, (P_OBS_NOISE << 24) | (uint32_t)(k / 4), key), z);
      for (int l = 0; l < 4 && k + l < md.dy; ++l) {
        const int o = md.obs_idx[k + l];
        float xo = x[0];
#pragma unroll
        for (int c = 1; c < D; ++c)
          if (o == c) xo = x[c];
        y[(size_t)(t - 1) * md.dy + k + l] = xo + obs_sd * z[l];
      }
    }
  }
}

inline dim3 vec_grid(const EnsDev &e) {
  return dim3((unsigned)((e.N + VEC_BLOCK - 1) / VEC_BLOCK), (unsigned)e.M);
}

}  // namespace

#define PF_DISPATCH_D(e, CALL3, CALL1) \
  do {                                  \
    if ((e).md.dx == 3) {               \
      CALL3;                            \
    } else {                            \
      CALL1;                            \
    }                                   \
  } while (0)

hipError_t launch_vec_init(const EnsDev &e, float *X, hipStream_t s) {
  PF_DISPATCH_D(e, (k_vec_init<3><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.key, e.N, X)),
                (k_vec_init<1><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.key, e.N, X)));
  return hipGetLastError();
}

hipError_t launch_vec_propagate(const EnsDev &e, int t, const float *Xin, const int32_t *anc,
                                float *Xout, float *lw, const float *y, hipStream_t s) {
  PF_DISPATCH_D(e,
                (k_vec_propagate<3><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.key, e.N, t, Xin, anc,
                                                                      Xout, lw, y)),
                (k_vec_propagate<1><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.key, e.N, t, Xin, anc,
                                                                      Xout, lw, y)));
  return hipGetLastError();
}

hipError_t launch_vec_prop_batched(int D, const int4 *d_tiles, int n_tiles, int tile_width,
                                  const FusedEns *d_ens, IvArg iv, int parity, int pending,
                                  hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (tile_width < 64 || tile_width > VEC_BLOCK || tile_width % 64) return hipErrorInvalidValue;
  if (D == 3)
    k_vec_prop_batched<3><<<n_tiles, tile_width, 0, s>>>(d_tiles, d_ens, iv, parity, pending);
  else
    k_vec_prop_batched<1><<<n_tiles, tile_width, 0, s>>>(d_tiles, d_ens, iv, parity, pending);
  return hipGetLastError();
}

hipError_t launch_vec_pilot(int D, const FusedEns *d_ens, int e, int M, int N, IvArg iv,
                            int parity, int pending, hipStream_t s) {
  const dim3 g((unsigned)((N + VEC_BLOCK - 1) / VEC_BLOCK), (unsigned)M);
  if (D == 3)
    k_vec_pilot<3><<<g, VEC_BLOCK, 0, s>>>(d_ens, e, iv, parity, pending);
  else
    k_vec_pilot<1><<<g, VEC_BLOCK, 0, s>>>(d_ens, e, iv, parity, pending);
  return hipGetLastError();
}

hipError_t launch_vec_loglik(const EnsDev &e, const float *X, const float *y, hipStream_t s) {
  PF_DISPATCH_D(e, (k_vec_loglik<3><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.N, X, y, e.lw)),
                (k_vec_loglik<1><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.md, e.N, X, y, e.lw)));
  return hipGetLastError();
}

hipError_t launch_vec_gather(const EnsDev &e, const float *Xin, float *Xout, hipStream_t s) {
  PF_DISPATCH_D(e, (k_vec_gather<3><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.N, e.A, Xin, Xout)),
                (k_vec_gather<1><<<vec_grid(e), VEC_BLOCK, 0, s>>>(e.N, e.A, Xin, Xout)));
  return hipGetLastError();
}

hipError_t launch_vec_estimate(const EnsDev &e, const float *Xpost, const float *Xpre,
                               const int32_t *anc, bool ensemble_mean, hipStream_t s) {
  dim3 g((unsigned)e.T, (unsigned)e.M);
  PF_DISPATCH_D(e,
                (k_vec_estimate_tiles<3><<<g, EST_THREADS, 0, s>>>(e.N, e.T, Xpost, Xpre, anc,
                                                                    e.lw, e.fstat, e.mpart,
                                                                    e.wpart)),
                (k_vec_estimate_tiles<1><<<g, EST_THREADS, 0, s>>>(e.N, e.T, Xpost, Xpre, anc,
                                                                    e.lw, e.fstat, e.mpart,
                                                                    e.wpart)));
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_combine_means(e, ensemble_mean, s);
}

hipError_t launch_vec_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                               hipStream_t s) {
  const Key key = make_key(seed);
  const float obs_sd = e.md.obs_sd;
  PF_DISPATCH_D(e, (k_vec_simulate<3><<<1, 64, 0, s>>>(e.md, key, T, obs_sd, xtrue, y)),
                (k_vec_simulate<1><<<1, 64, 0, s>>>(e.md, key, T, obs_sd, xtrue, y)));
  return hipGetLastError();
}

}  // namespace pfk
