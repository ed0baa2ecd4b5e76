// k_fhn_paper.hip -- the paper's modified stochastic FitzHugh-Nagumo network
// (Sec. 5.1, 5.2): a J x J grid of nodes (U, V) with a cubic reaction, the
// sum of the neighbours' U as coupling, periodic forcing of a corner block
// and random stimuli applied behind the waves.
//
// Particle state (float32, particle-major): the U plane [J*J], the V plane
// [J*J], then the ring of the last l0 stimulus events (slot n mod l0 holds
// the event of Euler step n: the centre node of the stimulated group, or
// -1), padded with -1 to a multiple of 4.
//
// One workgroup advances one particle at a time with the planes in LDS.
// Per Euler step n:
//   (a) the stimulus region: nodes whose U, or a 4-neighbour's U, lies in
//       (u-, u+) -- each thread flags its contiguous nodes, and one block
//       scan of the per-thread counts orders the region row-major;
//   (b) one Philox call (particle, filter, n, PROP | sub-block J*J/2): its
//       first uniform against eps decides the Bernoulli event, its second
//       picks the floor(u |S|)-th node of the region as the centre; the
//       thread whose range holds that node publishes it;
//   (c) the event enters the ring; a per-node count of the ring's coverage
//       (centre and its neighbours) is kept in LDS, so the stimulus of a
//       node is F~ when its count is positive (F~ min{1, sum Q});
//   (d) the Euler step of every node: U' = U + h (p3(U) - V) + h (c sum_nbr
//       U + m F + Psi) + sigma~ sqrt(h) z, V' = V + h (b0 U + b1 V + b2),
//       the normals of node pair p from the FH-N grid layout (call (particle,
//       filter, n, PROP | p): lanes 0, 1 for node 2p, lanes 2, 3 for 2p + 1).
// The first read goes through the ancestors (fused gather); the last step
// ends with the log-likelihood of the observed U nodes.
#include "pf_internal.h"

namespace pfk {
namespace {

constexpr int FP_THREADS = 256;

struct FhnpLds {
  float *u, *un, *v;  // [nn] each
  int *inr, *cov;     // [nn] each
  int *ring;          // [32]
  int *scan;          // [FP_THREADS / 64 + 4]: wave sums, then broadcast slots
};

__device__ __forceinline__ FhnpLds fhnp_lds(int nn) {
  extern __shared__ float fp_lds[];
  FhnpLds L;
  L.u = fp_lds;
  L.un = L.u + nn;
  L.v = L.un + nn;
  L.inr = (int *)(L.v + nn);
  L.cov = L.inr + nn;
  L.ring = L.cov + nn;
  L.scan = L.ring + 32;
  return L;
}

// the centre node and its neighbours inside the grid: +d to the coverage
__device__ __forceinline__ void cover(int *cov, int J, int c, int d) {
  if (c < 0) return;
  const int i = c / J, j = c - i * J;
  cov[c] += d;
  if (i > 0) cov[c - J] += d;
  if (i < J - 1) cov[c + J] += d;
  if (j > 0) cov[c - 1] += d;
  if (j < J - 1) cov[c + 1] += d;
}

__device__ __forceinline__ bool in_band(const ModelDev &md, float u) {
  return u > md.stim_lo && u < md.stim_hi;
}

// Node range of a thread: P consecutive nodes, P even (whole noise pairs).
__device__ __forceinline__ int fhnp_per_thread(int nn) {
  return 2 * ((nn + 2 * FP_THREADS - 1) / (2 * FP_THREADS));
}

// S Euler steps n0 .. n0 + S - 1 of the particle in LDS (u, v, ring, cov).
// c0, c1, purpose: its Philox stream.  Leaves the state in L.u, L.v, L.ring.
// PILOT: the noise-free continuation (the auxiliary filter's pilot): no new
// stimulus event and no noise; the ring's active stimuli and the forcing act.
template <bool PILOT>
__device__ void fhnp_steps(const ModelDev &md, Key key, uint32_t purpose, uint32_t c0,
                           uint32_t c1, int n0, FhnpLds &L) {
  const int J = md.J, nn = J * J, tid = threadIdx.x;
  const int P = fhnp_per_thread(nn), k0 = tid * P;
  const int lane = tid & 63, wid = tid >> 6;
  for (int st = 0; st < md.S; ++st) {
    const uint32_t n = (uint32_t)(n0 + st);
    if (PILOT) {
      if (tid == 0) L.scan[FP_THREADS / 64 + 1] = -1;
      __syncthreads();
    } else {
      // (a) stimulus region
      for (int e = 0; e < P; ++e) {
        const int k = k0 + e;
        if (k < nn) L.inr[k] = in_band(md, L.u[k]) ? 1 : 0;
      }
      __syncthreads();
      int cnt = 0;
      for (int e = 0; e < P; ++e) {
        const int k = k0 + e;
        if (k < nn) {
          const int i = k / J, j = k - i * J;
          const int r = L.inr[k] | (i > 0 ? L.inr[k - J] : 0) | (i < J - 1 ? L.inr[k + J] : 0) |
                        (j > 0 ? L.inr[k - 1] : 0) | (j < J - 1 ? L.inr[k + 1] : 0);
          cnt += r;
        }
      }
      // exclusive scan of the counts over the workgroup
      int inc = cnt;
  #pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      if (lane == 63) L.scan[wid] = inc;
      __syncthreads();
      int off = inc - cnt, total = 0;
      for (int w = 0; w < FP_THREADS / 64; ++w) {
        if (w < wid) off += L.scan[w];
        total += L.scan[w];
      }
      // (b) the Bernoulli event and its centre
      if (tid == 0) {
        const uint4 r = philox(c0, c1, n, (purpose << 24) | (uint32_t)(nn / 2), key);
        int kth = -1;
        if (total > 0 && u01d(r.x) < md.stim_eps) {
          kth = (int)floor(u01d(r.y) * (double)total);
          kth = min(kth, total - 1);
        }
        L.scan[FP_THREADS / 64] = kth;
        L.scan[FP_THREADS / 64 + 1] = -1;
      }
      __syncthreads();
      const int kth = L.scan[FP_THREADS / 64];
      if (kth >= off && kth < off + cnt) {
        int want = kth - off;
        for (int e = 0; e < P; ++e) {
          const int k = k0 + e;
          if (k < nn) {
            const int i = k / J, j = k - i * J;
            const int r = L.inr[k] | (i > 0 ? L.inr[k - J] : 0) | (i < J - 1 ? L.inr[k + J] : 0) |
                          (j > 0 ? L.inr[k - 1] : 0) | (j < J - 1 ? L.inr[k + 1] : 0);
            if (r && want-- == 0) L.scan[FP_THREADS / 64 + 1] = k;
          }
        }
      }
      __syncthreads();
    }
    // (c) the ring and the coverage counts
    if (tid == 0) {
      const int slot = (int)(n % (uint32_t)md.stim_l0);
      const int ev = L.scan[FP_THREADS / 64 + 1];
      cover(L.cov, J, L.ring[slot], -1);
      L.ring[slot] = ev;
      cover(L.cov, J, ev, +1);
    }
    __syncthreads();
    // (d) Euler step of this thread's node pairs
    const bool forcing = (int)(n % (uint32_t)md.force_period) < md.force_width;
    for (int e = 0; e < P; e += 2) {
      const int k = k0 + e;
      if (k >= nn) break;
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (!PILOT) normals4(philox(c0, c1, n, (purpose << 24) | (uint32_t)(k >> 1), key), z);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int kk = k + q;
        const int i = kk / J, j = kk - i * J;
        float sum = 0.f;
        if (i > 0) sum += L.u[kk - J];
        if (i < J - 1) sum += L.u[kk + J];
        if (j > 0) sum += L.u[kk - 1];
        if (j < J - 1) sum += L.u[kk + 1];
        const float u = L.u[kk], v = L.v[kk];
        const float psi = L.cov[kk] > 0 ? md.stim_amp : 0.f;
        const float mf = (forcing && i < 2 && j < 2) ? md.stim_amp : 0.f;
        const float p3 = md.p0 * u - u * u * u;
        const float un = (u + md.h * (p3 - v)) + md.h * (md.p1 * sum + mf + psi);
        L.un[kk] = fmaf(md.sq0, z[2 * q], un);
        const float vn = v + md.h * (md.p2 * u + md.p3 * v + md.stim_b2);
        L.v[kk] = fmaf(md.sq1, z[2 * q + 1], vn);
      }
    }
    __syncthreads();
    float *tmp = L.u;
    L.u = L.un;
    L.un = tmp;
  }
}

// Load the particle (U, V, ring) into LDS and build the coverage counts.
__device__ __forceinline__ void fhnp_load(const ModelDev &md, const float *x, FhnpLds &L) {
  const int nn = md.J * md.J, l0 = md.stim_l0;
  for (int k = threadIdx.x; k < nn; k += FP_THREADS) {
    L.u[k] = x[k];
    L.v[k] = x[nn + k];
    L.cov[k] = 0;
  }
  if (threadIdx.x < 32) L.ring[threadIdx.x] = threadIdx.x < l0 ? (int)x[2 * nn + threadIdx.x] : -1;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int l = 0; l < l0; ++l) cover(L.cov, md.J, L.ring[l], +1);
  __syncthreads();
}

__device__ __forceinline__ void fhnp_store(const ModelDev &md, float *x, const FhnpLds &L) {
  const int nn = md.J * md.J, ring = md.dx - 2 * nn;
  for (int k = threadIdx.x; k < nn; k += FP_THREADS) {
    x[k] = L.u[k];
    x[nn + k] = L.v[k];
  }
  if (threadIdx.x < ring) x[2 * nn + threadIdx.x] = threadIdx.x < md.stim_l0 ? (float)L.ring[threadIdx.x] : -1.f;
}

// Interval t of every particle of one ensemble (fused path): read through
// the ancestors when `pending`, S steps, state out, log-likelihood.
__global__ void __launch_bounds__(FP_THREADS)
k_fhnp_steps(const FusedEns *__restrict__ ens, int e, IvArg iv, int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const FusedEns &E = ens[e];
  const ModelDev md = E.md;
  const int nn = md.J * md.J, dx = md.dx, N = E.N, MN = E.M * N;
  FhnpLds L = fhnp_lds(nn);
  const float *Xin = parity ? E.X1 : E.X0;
  float *Xout = parity ? E.X0 : E.X1;
  for (int p = blockIdx.x; p < MN; p += gridDim.x) {
    const int m = p / N, i = p - m * N;
    // (an auxiliary filter's particles always come through the ancestors its
    // first stage has just drawn)
    const bool thru = pending || E.apf;
    const int src = thru ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
    fhnp_load(md, Xin + ((size_t)m * N + src) * dx, L);
    fhnp_steps<false>(md, E.key, P_PROP, (uint32_t)i, (uint32_t)m, (t - 1) * md.S, L);
    fhnp_store(md, Xout + ((size_t)m * N + i) * dx, L);
    if (y) {
      float acc = 0.f;
      for (int k = threadIdx.x; k < md.dy; k += FP_THREADS) {
        const float r = gptr(y)[E.yoff + k] - L.u[gptr(md.obs_idx)[k]];
        acc = fmaf(r, r, acc);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) L.scan[threadIdx.x >> 6] = __float_as_int(acc);
      __syncthreads();
      if (threadIdx.x == 0) {
        float a = 0.f;
        for (int w = 0; w < FP_THREADS / 64; ++w) a += __int_as_float(L.scan[w]);
        float l = -a * md.inv2var;
        // auxiliary filter: divided by the pilot likelihood of the ancestor
        if (E.apf) l -= gptr(E.lpil)[(size_t)m * N + src];
        gptr(E.lw)[(size_t)m * N + i] = l == l ? l : -INFINITY;
      }
    }
    __syncthreads();
  }
}

// Auxiliary filters: the pilot of every particle -- S noise-free steps
// without new stimuli -- its log-likelihood, kept for the second stage, and
// the first-stage log-weight lwc + log g(y | mu).
__global__ void __launch_bounds__(FP_THREADS)
k_fhnp_pilot(const FusedEns *__restrict__ ens, int e, IvArg iv, int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const FusedEns &E = ens[e];
  const ModelDev md = E.md;
  const int nn = md.J * md.J, dx = md.dx, N = E.N, MN = E.M * N;
  FhnpLds L = fhnp_lds(nn);
  const float *Xin = parity ? E.X1 : E.X0;
  for (int p = blockIdx.x; p < MN; p += gridDim.x) {
    const int m = p / N, i = p - m * N;
    const int src = pending ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
    fhnp_load(md, Xin + ((size_t)m * N + src) * dx, L);
    fhnp_steps<true>(md, E.key, P_PROP, (uint32_t)i, (uint32_t)m, (t - 1) * md.S, L);
    float acc = 0.f;
    for (int k = threadIdx.x; k < md.dy; k += FP_THREADS) {
      const float r = gptr(y)[E.yoff + k] - L.u[gptr(md.obs_idx)[k]];
      acc = fmaf(r, r, acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) L.scan[threadIdx.x >> 6] = __float_as_int(acc);
    __syncthreads();
    if (threadIdx.x == 0) {
      float a = 0.f;
      for (int w = 0; w < FP_THREADS / 64; ++w) a += __int_as_float(L.scan[w]);
      float pl = -a * md.inv2var;
      pl = pl == pl ? pl : -INFINITY;
      const size_t o = (size_t)m * N + i;
      gptr(E.lpil)[o] = pl;
      const float lam = pl + gptr(E.lwc)[o];
      gptr(E.lw)[o] = lam == lam ? lam : -INFINITY;
    }
    __syncthreads();
  }
}

// Truth path and observations on the truth stream: one workgroup, T
// intervals of S steps from x_0 ~ tau_0.
__global__ void __launch_bounds__(FP_THREADS)
k_fhnp_simulate(ModelDev md, Key key, int T, float *__restrict__ xtrue, float *__restrict__ y) {
  const int nn = md.J * md.J, dx = md.dx;
  FhnpLds L = fhnp_lds(nn);
  for (int s = threadIdx.x; s < dx; s += FP_THREADS) {
    float z[4];
    normals4(philox(0u, TRUTH_STREAM, 0u, (P_TRUTH_INIT << 24) | (uint32_t)(s >> 2), key), z);
    xtrue[s] = md.prior_mean[s] + md.prior_sd[s] * z[s & 3];
  }
  __syncthreads();
  fhnp_load(md, xtrue, L);
  for (int t = 1; t <= T; ++t) {
    fhnp_steps<false>(md, key, P_TRUTH_NOISE, 0u, TRUTH_STREAM, (t - 1) * md.S, L);
    fhnp_store(md, xtrue + (size_t)t * dx, L);
    for (int k4 = threadIdx.x; 4 * k4 < md.dy; k4 += FP_THREADS) {
      float z[4];
      normals4(philox(0u, TRUTH_STREAM, (uint32_t)t, (P_OBS_NOISE << 24) | (uint32_t)k4, key), z);
      for (int l = 0; l < 4 && 4 * k4 + l < md.dy; ++l)
        y[(size_t)(t - 1) * md.dy + 4 * k4 + l] = L.u[md.obs_idx[4 * k4 + l]] + md.obs_sd * z[l];
    }
    __syncthreads();
  }
}

size_t fhnp_lds_bytes(int J) {
  const size_t nn = (size_t)J * J;
  return sizeof(float) * 3 * nn + sizeof(int) * (2 * nn + 32 + FP_THREADS / 64 + 4);
}

}  // namespace

hipError_t launch_fhnp_steps(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s) {
  int per_cu = 0, dev = 0, cus = 256;
  const size_t lds = fhnp_lds_bytes(J);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fhnp_steps, FP_THREADS,
                                                   lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int blocks = std::min(M * N, per_cu * cus);
  k_fhnp_steps<<<blocks, FP_THREADS, lds, s>>>(d_ens, e, iv, parity, pending);
  return hipGetLastError();
}

hipError_t launch_fhnp_pilot(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s) {
  int per_cu = 0, dev = 0, cus = 256;
  const size_t lds = fhnp_lds_bytes(J);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fhnp_pilot, FP_THREADS,
                                                   lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int blocks = std::min(M * N, per_cu * cus);
  k_fhnp_pilot<<<blocks, FP_THREADS, lds, s>>>(d_ens, e, iv, parity, pending);
  return hipGetLastError();
}

hipError_t launch_fhnp_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                                hipStream_t s) {
  k_fhnp_simulate<<<1, FP_THREADS, fhnp_lds_bytes(e.md.J), s>>>(e.md, make_key(seed), T, xtrue,
                                                                 y);
  return hipGetLastError();
}

}  // namespace pfk
