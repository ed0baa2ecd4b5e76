// k_grid.hip -- kernels of the FitzHugh-Nagumo grid model (J x J nodes, two
// variables per node, particle-major state [M][N][2][J][J]: the v plane then
// the w plane of each particle, contiguous).
//
// A thread handles float4 slots s of a particle (nodes 4s .. 4s+3 in
// row-major order): v and w of its nodes live in registers, and the v plane
// is staged in LDS because the 5-point Laplacian reads the neighbours' v.
// The streaming kernel gives a workgroup one particle (slots s = t,
// t + blockDim, ...); the blocked kernel a few particles of one ensemble.
//   - k_grid_steps: every Euler step of the interval with the plane resident
//     in LDS (temporal blocking: the state crosses HBM once per interval);
//     the first read goes through the ancestor index (fused gather) and the
//     last step also produces the log-weight (fused weighting).
//   - k_grid_stream_step: one Euler step per launch, state read from and
//     written to HBM (16 bytes per node-step).
// Both share grid_euler(): drift v(v-a)(1-v) - w + D lap(v), eps (v - gam w),
// Euler-Maruyama with the increments of an interval summed in an FP32 offset
// from its start state (the blocked and the simulation kernels; compensated
// sums where several particles share a workgroup, whose registers are
// fewer; a plain update for the streaming kernel's single step), the noise
// of nodes 2p, 2p+1 from the Philox call of node pair p at step n.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "pf_internal.h"

namespace pfk {
namespace {

constexpr int GB = 256;  // workgroup size of the element-wise grid kernels
// The streaming and simulation kernels run 64 * ceil(slots / (64 * SPT))
// threads with SPT float4 slots each (slots = J*J/4); J <= 64 needs at most
// 1024 slots.

typedef float f4v __attribute__((ext_vector_type(4)));
// streaming access: the state of a step is touched once and exceeds every cache
__device__ __forceinline__ float4 ld_stream(const float4 *p) {
  const f4v v = __builtin_nontemporal_load((const f4v *)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float4 *p, const float4 &a) {
  f4v v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, (f4v *)p);
}

struct Slot4 {
  // state of 4 nodes, the sums of their increments since the interval's
  // start (or the compensation terms of compensated sums), and the start
  // state
  float4 v, w, dv, dw, v0, w0;
  __device__ void start(float4 a, float4 b) {
    v = v0 = a;
    w = w0 = b;
    dv = dw = make_float4(0.f, 0.f, 0.f, 0.f);
  }
};

__device__ __forceinline__ float get(const float4 &a, int e) {
  return e == 0 ? a.x : e == 1 ? a.y : e == 2 ? a.z : a.w;
}
__device__ __forceinline__ void set(float4 &a, int e, float x) {
  if (e == 0) a.x = x; else if (e == 1) a.y = x; else if (e == 2) a.z = x; else a.w = x;
}

// LDS indices of the up / down / left / right neighbours of the 4 nodes of
// slot s; a neighbour outside the grid points at the node itself, so its
// term v_nbr - v is exactly +0 and the sum equals the truncated one.
struct Nbr4 {
  int u[4], d[4], l[4], r[4];
};

__device__ __forceinline__ Nbr4 neighbours(int J, int s) {
  Nbr4 n;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * s + e;
    const int i = k / J, j = k - i * J;
    n.u[e] = i > 0 ? k - J : k;
    n.d[e] = i < J - 1 ? k + J : k;
    n.l[e] = j > 0 ? k - 1 : k;
    n.r[e] = j < J - 1 ? k + 1 : k;
  }
  return n;
}

// Neighbour addresses of slot s when J is a multiple of 4, so that the
// slot's 4 nodes lie in one row: the 4 nodes above and the 4 below as one
// 16-byte read each (the slot itself on the top / bottom row: no-flux), the
// left neighbour of the first node and the right neighbour of the last (the
// node itself at the left / right edge); the inner left and right
// neighbours are the slot's own values.
struct Row4 {
  int u, d, l, r;
};

__device__ __forceinline__ Row4 row4_addrs(int J, int s) {
  const int k = 4 * s, i = k / J, j = k - i * J;
  return Row4{i > 0 ? k - J : k, i < J - 1 ? k + J : k, j > 0 ? k - 1 : k,
              j + 3 < J - 1 ? k + 4 : k + 3};
}

// v of the up, down, left and right neighbours of the slot's 4 nodes
__device__ __forceinline__ void fetch_nbrs(const Nbr4 &nb, const float *vs, const float4 &,
                                           float vu[4], float vd[4], float vl[4], float vr[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    vu[e] = vs[nb.u[e]];
    vd[e] = vs[nb.d[e]];
    vl[e] = vs[nb.l[e]];
    vr[e] = vs[nb.r[e]];
  }
}
__device__ __forceinline__ void fetch_nbrs(const Row4 &nb, const float *vs, const float4 &v,
                                           float vu[4], float vd[4], float vl[4], float vr[4]) {
  const float4 a = *(const float4 *)(vs + nb.u), b = *(const float4 *)(vs + nb.d);
  const float L = vs[nb.l], R = vs[nb.r];
  vu[0] = a.x; vu[1] = a.y; vu[2] = a.z; vu[3] = a.w;
  vd[0] = b.x; vd[1] = b.y; vd[2] = b.z; vd[3] = b.w;
  vl[0] = L;   vl[1] = v.x; vl[2] = v.y; vl[3] = v.z;
  vr[0] = v.y; vr[1] = v.z; vr[2] = v.w; vr[3] = R;
}

// One Euler-Maruyama step of the 4 nodes of slot s (nodes 4s .. 4s+3), reading
// neighbour v values from the LDS plane vs (which holds S.v for this slot).
// Returns the new state in S.  MODE: the increments summed in an offset from
// the interval's start state S.v0, S.w0 (EULER_OFFSET), compensated sums
// with S.dv, S.dw the compensation terms (EULER_KAHAN), or a single step
// from S.v, S.w (EULER_SINGLE).
constexpr int EULER_OFFSET = 0, EULER_KAHAN = 1, EULER_SINGLE = 2;
template <int MODE, class NB>
__device__ __forceinline__ void grid_euler(const ModelDev &md, Key key, uint32_t purpose,
                                           uint32_t c0, uint32_t c1, uint32_t n, int s,
                                           const NB &nb, const float *vs, Slot4 &S) {
  const uint4 ra = philox<4, 3>(c0, c1, n, (purpose << 24) | (uint32_t)(2 * s), key);
  const uint4 rb = philox<4, 3>(c0, c1, n, (purpose << 24) | (uint32_t)(2 * s + 1), key);
  float za[4], zb[4];
  normals4(ra, za);
  normals4(rb, zb);
  // node 4s+e: pair 2s + e/2; lanes (0,1) for the even node, (2,3) the odd
  const float zv[4] = {za[0], za[2], zb[0], zb[2]};
  const float zw[4] = {za[1], za[3], zb[1], zb[3]};
  float vu[4], vd[4], vl[4], vr[4];
  fetch_nbrs(nb, vs, S.v, vu, vd, vl, vr);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float c = get(S.v, e), w = get(S.w, e);
    const float lap = (((vu[e] - c) + (vd[e] - c)) + (vl[e] - c)) + (vr[e] - c);
    float nv, nw;
    if constexpr (MODE == EULER_SINGLE) {
      float dv = 0.f, dw = 0.f;
      fhn_node_step_off<false>(md, c, w, lap, zv[e], zw[e], 0.f, 0.f, c, w, nv, nw, dv, dw);
    } else {
      float dv = get(S.dv, e), dw = get(S.dw, e);
      if constexpr (MODE == EULER_OFFSET)
        fhn_node_step_off<false>(md, c, w, lap, zv[e], zw[e], 0.f, 0.f, get(S.v0, e),
                                 get(S.w0, e), nv, nw, dv, dw);
      else
        fhn_node_step<false>(md, c, w, lap, zv[e], zw[e], 0.f, 0.f, nv, nw, dv, dw);
      set(S.dv, e, dv);
      set(S.dw, e, dw);
    }
    set(S.v, e, nv);
    set(S.w, e, nw);
  }
}

// -(1/(2 sigma^2)) sum_k (y_k - v[obs_k])^2 from the LDS plane (workgroup sum)
__device__ __forceinline__ float grid_loglik(const ModelDev &md, const float *vs, const float *y,
                                             float *shf) {
  float acc = 0.f;
  for (int k = threadIdx.x; k < md.dy; k += blockDim.x) {
    const float r = gptr(y)[k] - vs[gptr(md.obs_idx)[k]];
    acc = fmaf(r, r, acc);
  }
  // block sum in FP32 (fixed order over waves)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) shf[threadIdx.x >> 6] = acc;
  __syncthreads();
  float tot = 0.f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += shf[i];
  const float lw = -tot * md.inv2var;
  return (lw == lw) ? lw : -INFINITY;
}

// -(1/(2 sigma^2)) sum_k (y_k - v[obs_k])^2 of one particle by one wavefront:
// lane l sums the terms k = l, l + 64, ... in order, then a butterfly over
// the 64 lanes (every lane returns the total).
__device__ __forceinline__ float wave_loglik(const ModelDev &md, const float *vs, const float *y,
                                             int lane) {
  float acc = 0.f;
  for (int k = lane; k < md.dy; k += 64) {
    const float r = gptr(y)[k] - vs[gptr(md.obs_idx)[k]];
    acc = fmaf(r, r, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  const float lw = -acc * md.inv2var;
  return (lw == lw) ? lw : -INFINITY;
}

// Interval of S steps per particle with the v plane resident in LDS, over a
// table of {ensemble, filter, particle, -} entries of grid ensembles that
// share J (one launch serves a whole batch of them).  A workgroup holds ppb
// particles of one ensemble at a time -- thread t works on slot t % slots of
// particle t / slots -- so that ppb * slots threads fill whole wavefronts
// (J = 40: 2 x 400 slots in 832 threads; J = 20: 5 x 100 in 512).  Every
// ensemble's entries are padded to a multiple of ppb with ensemble -1.
// MULTI = false is the ppb = 1 form, whose particle indices stay uniform
// (scalar registers).  ROW4: J is a multiple of 4 (neighbours by Row4).
template <bool MULTI, bool ROW4>
__device__ __forceinline__ void grid_steps(const int4 *__restrict__ ptab, int n_p,
                                           const FusedEns *__restrict__ ens, IvArg iv, int parity,
                                           int pending, int J, int ppb_arg) {
  const int t = iv_t(iv);
  const float *yb = iv_y(iv, t);
  extern __shared__ float planes[];  // [ppb][J*J] v planes
  const int ppb = MULTI ? ppb_arg : 1;
  const int nn = J * J, slots = nn / 4, dx = 2 * nn;
  const int q = MULTI ? (int)threadIdx.x / slots : 0, sl = (int)threadIdx.x - q * slots;
  const bool has_slot = MULTI ? q < ppb : sl < slots;
  float *vs = planes + (has_slot ? q : 0) * nn;
  std::conditional_t<ROW4, Row4, Nbr4> nb;
  if constexpr (ROW4)
    nb = row4_addrs(J, has_slot ? sl : 0);
  else
    nb = neighbours(J, has_slot ? sl : 0);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int p0 = blockIdx.x * ppb; p0 < n_p; p0 += gridDim.x * ppb) {
    // the first entry of a group is never padding
    const FusedEns &E = ens[ptab[p0].x];
    const ModelDev md = E.md;
    const Key key = E.key;
    const int N = E.N;
    int4 pt = make_int4(-1, 0, 0, 0);
    if (!MULTI) pt = ptab[p0];
    else if (has_slot) pt = ptab[p0 + q];
    const bool on = MULTI ? pt.x >= 0 : has_slot;
    const int m = pt.y, i = pt.z;
    const float *Xin = parity ? E.X1 : E.X0;
    float *Xout = parity ? E.X0 : E.X1;
    Slot4 S;
    // (an auxiliary filter's particles always come through the ancestors its
    // first stage has just drawn)
    const bool thru = pending || E.apf;
    if (on) {
      const int src = thru ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
      const gmem<f4v> *in = gptr((const f4v *)(Xin + ((size_t)m * N + src) * dx));
      const f4v a = in[sl], b = in[slots + sl];
      S.start(make_float4(a.x, a.y, a.z, a.w), make_float4(b.x, b.y, b.z, b.w));
      *(float4 *)(vs + 4 * sl) = S.v;
    }
    __syncthreads();
    const int n0 = (t - 1) * md.S;
    for (int st = 0; st < md.S; ++st) {
      if (on)
        grid_euler<MULTI ? EULER_KAHAN : EULER_OFFSET>(md, key, P_PROP, (uint32_t)i, (uint32_t)m,
                                                       (uint32_t)(n0 + st), sl, nb, vs, S);
      __syncthreads();
      if (on) *(float4 *)(vs + 4 * sl) = S.v;
      __syncthreads();
    }
    if (on) {
      gmem<f4v> *out = gptr((f4v *)(Xout + ((size_t)m * N + i) * dx));
      out[sl] = f4v{S.v.x, S.v.y, S.v.z, S.v.w};
      out[slots + sl] = f4v{S.w.x, S.w.y, S.w.z, S.w.w};
    }
    if (yb) {
      // one wavefront per particle of the group
      for (int qq = wid; qq < ppb; qq += nwaves) {
        const int4 pq = ptab[p0 + qq];
        if (pq.x >= 0) {
          float l = wave_loglik(md, planes + qq * nn, yb + E.yoff, lane);
          // auxiliary filter: divided by the pilot likelihood of the ancestor
          if (E.apf && lane == 0) {
            const int a = min(max(gptr(E.A)[(size_t)pq.y * N + pq.z], 0), N - 1);
            l -= gptr(E.lpil)[(size_t)pq.y * N + a];
            l = l == l ? l : -INFINITY;
          }
          if (lane == 0) gptr(E.lw)[(size_t)pq.y * N + pq.z] = l;
        }
      }
    }
    __syncthreads();
  }
}

template <bool ROW4>
__global__ void __launch_bounds__(1024)
k_grid_steps(const int4 *__restrict__ ptab, int n_p, const FusedEns *__restrict__ ens, IvArg iv,
             int parity, int pending, int J) {
  grid_steps<false, ROW4>(ptab, n_p, ens, iv, parity, pending, J, 1);
}

// (at most 64 VGPRs, 8 wavefronts per SIMD: the few values it spills are
// reloaded once per particle group, outside the Euler steps)
template <bool ROW4>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_grid_steps_multi(const int4 *__restrict__ ptab, int n_p, const FusedEns *__restrict__ ens,
                   IvArg iv, int parity, int pending, int J, int ppb) {
  grid_steps<true, ROW4>(ptab, n_p, ens, iv, parity, pending, J, ppb);
}

// One Euler step n of every particle, state through HBM.
template <int SPT>
__global__ void __launch_bounds__(1024)
k_grid_stream_step(ModelDev md, Key key, int M, int N, int n, const float *Xin,
                   const int32_t *__restrict__ anc, float *Xout,
                   float *__restrict__ lw, const float *__restrict__ y) {
  // Xin may equal Xout (in-place step): each workgroup reads its whole
  // particle before the barrier and writes it after.  The workgroup's next
  // two particles are in flight into registers (two sets, alternating) while
  // the current one computes: a particle's load is issued two particles
  // ahead, as soon as its register set has been taken.
  extern __shared__ float vs[];
  const int J = md.J, nn = J * J, slots = nn / 4, dx = 2 * nn, MN = M * N, G = gridDim.x;
  float *shf = vs + nn;
  Nbr4 nb[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) nb[q] = neighbours(J, min((int)(threadIdx.x + q * blockDim.x), slots - 1));
  float4 av[SPT], aw[SPT], bv[SPT], bw[SPT];
  auto load = [&](int p, float4 (&nv)[SPT], float4 (&nw)[SPT]) {
    const int m = p / N, i = p - m * N;
    const int src = anc ? min(max(anc[(size_t)m * N + i], 0), N - 1) : i;
    const float4 *in = (const float4 *)(Xin + ((size_t)m * N + src) * dx);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int s = threadIdx.x + q * blockDim.x;
      if (s < slots) {
        nv[q] = ld_stream(in + s);
        nw[q] = ld_stream(in + slots + s);
      }
    }
  };
  auto particle = [&](int p, float4 (&nv)[SPT], float4 (&nw)[SPT]) {
    const int m = p / N, i = p - m * N;
    Slot4 S[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int s = threadIdx.x + q * blockDim.x;
      if (s < slots) {
        S[q].start(nv[q], nw[q]);
        *(float4 *)(vs + 4 * s) = S[q].v;
      }
    }
    __syncthreads();
    if (p + 2 * G < MN) load(p + 2 * G, nv, nw);
    float4 *out = (float4 *)(Xout + ((size_t)m * N + i) * dx);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int s = threadIdx.x + q * blockDim.x;
      if (s < slots) {
        grid_euler<EULER_SINGLE>(md, key, P_PROP, (uint32_t)i, (uint32_t)m, (uint32_t)n, s, nb[q], vs,
                                 S[q]);
        st_stream(out + s, S[q].v);
        st_stream(out + slots + s, S[q].w);
      }
    }
    if (lw) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int s = threadIdx.x + q * blockDim.x;
        if (s < slots) *(float4 *)(vs + 4 * s) = S[q].v;
      }
      __syncthreads();
      const float l = grid_loglik(md, vs, y, shf);
      if (threadIdx.x == 0) lw[(size_t)m * N + i] = l;
    }
    __syncthreads();
  };
  const int p0 = blockIdx.x;
  if (p0 < MN) load(p0, av, aw);
  if (p0 + G < MN) load(p0 + G, bv, bw);
  for (int p = p0; p < MN; p += 2 * G) {
    particle(p, av, aw);
    if (p + G < MN) particle(p + G, bv, bw);
  }
}

// Auxiliary filters: the pilot of one particle per workgroup -- its
// noise-free S-step Euler path on the grid (v planes double-buffered in LDS,
// w in LDS, updated in place: a node's w step reads only its own v and w)
// -- its log-likelihood, kept for the second stage, and the first-stage
// log-weight lwc + log g(y | mu).
constexpr int PILOT_THREADS = 256;
__global__ void __launch_bounds__(PILOT_THREADS)
k_grid_pilot(const FusedEns *__restrict__ ens, int e, IvArg iv, int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const FusedEns &E = ens[e];
  const ModelDev md = E.md;
  const int J = md.J, nn = J * J, N = E.N;
  const int p = blockIdx.x, m = p / N, i = p - m * N;
  extern __shared__ float sh[];
  float *v = sh, *vn = sh + nn, *w = sh + 2 * nn, *red = sh + 3 * nn;
  const int src = pending ? min(max(gptr(E.A)[(size_t)m * N + i], 0), N - 1) : i;
  const gmem<float> *x = gptr((parity ? E.X1 : E.X0) + ((size_t)m * N + src) * 2 * nn);
  for (int n = threadIdx.x; n < nn; n += PILOT_THREADS) {
    v[n] = x[n];
    w[n] = x[nn + n];
  }
  __syncthreads();
  const float a = md.p0, D = md.p1, eps = md.p2, gam = md.p3, h = md.h;
  for (int st = 0; st < md.S; ++st) {
    for (int n = threadIdx.x; n < nn; n += PILOT_THREADS) {
      const int r = n / J, c = n - r * J;
      const float vc = v[n], wc = w[n];
      float lap = 0.f;
      if (r > 0) lap += v[n - J] - vc;
      if (r < J - 1) lap += v[n + J] - vc;
      if (c > 0) lap += v[n - 1] - vc;
      if (c < J - 1) lap += v[n + 1] - vc;
      const float fv = vc * (vc - a) * (1.f - vc) - wc + D * lap;
      const float fw = eps * (vc - gam * wc);
      vn[n] = fmaf(h, fv, vc);
      w[n] = fmaf(h, fw, wc);
    }
    __syncthreads();
    float *tmp = v;
    v = vn;
    vn = tmp;
  }
  float acc = 0.f;
  for (int k = threadIdx.x; k < md.dy; k += PILOT_THREADS) {
    const float rr = gptr(y)[E.yoff + k] - v[gptr(md.obs_idx)[k]];
    acc = fmaf(rr, rr, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.f;
    for (int k = 0; k < PILOT_THREADS / 64; ++k) tot += red[k];
    float pl = -tot * md.inv2var;
    pl = pl == pl ? pl : -INFINITY;
    const size_t o = (size_t)m * N + i;
    gptr(E.lpil)[o] = pl;
    const float lam = pl + gptr(E.lwc)[o];
    gptr(E.lw)[o] = lam == lam ? lam : -INFINITY;
  }
}

// Prior draw: state index s of particle i uses Philox (i, m, 0, INIT | s/4).
__global__ void __launch_bounds__(GB)
k_grid_init(ModelDev md, Key key, int N, float *__restrict__ X) {
  const int dx = md.dx, p = blockIdx.x;  // p = m * N + i
  const int m = p / N, i = p - m * N;
  float *x = X + (size_t)p * dx;
  for (int g = threadIdx.x; 4 * g < dx; g += GB) {  // group of 4 states
    float z[4];
    normals4(philox((uint32_t)i, (uint32_t)m, 0u, (P_INIT << 24) | (uint32_t)g, key), z);
    for (int l = 0; l < 4 && 4 * g + l < dx; ++l)
      x[4 * g + l] = md.prior_mean[4 * g + l] + md.prior_sd[4 * g + l] * z[l];
  }
}

// log-weights of every particle from its stored state (plain path).
__global__ void __launch_bounds__(GB)
k_grid_loglik(ModelDev md, int M, int N, const float *__restrict__ X, const float *__restrict__ y,
              float *__restrict__ lw) {
  const int p = blockIdx.x * GB + threadIdx.x;
  if (p >= M * N) return;
  const float *v = X + (size_t)p * md.dx;
  float acc = 0.f;
  for (int k = 0; k < md.dy; ++k) {
    const float r = y[k] - v[md.obs_idx[k]];
    acc = fmaf(r, r, acc);
  }
  const float l = -acc * md.inv2var;
  lw[p] = (l == l) ? l : -INFINITY;
}

// x'[m][k] = xbar[m][a_k]: float4 block copies.
__global__ void __launch_bounds__(GB)
k_grid_gather(int N, int dx4, const int32_t *__restrict__ A, const float4 *__restrict__ Xin,
              float4 *__restrict__ Xout) {
  const int p = blockIdx.x;  // m * N + k
  const int m = p / N;
  const int a = min(max(A[p], 0), N - 1);
  const float4 *src = Xin + ((size_t)m * N + a) * dx4;
  float4 *dst = Xout + (size_t)p * dx4;
  for (int g = threadIdx.x; g < dx4; g += GB) dst[g] = src[g];
}

// Partial sums over a chunk of particles of one filter, per state element:
// post-resampling sum_i n_i xbar_i (n_i offspring counts) and weighted
// sum_i w_i xbar_i, both in FP64.  Grid: (state groups, chunks, M).
constexpr int EST_CHUNK = 64;
__global__ void __launch_bounds__(GB)
k_grid_estimate_part(int N, int dx4, const float4 *__restrict__ Xb,
                     const int32_t *__restrict__ cnt, const float *__restrict__ lw,
                     const double *__restrict__ fstat, double *__restrict__ part) {
  // the chunk's offspring counts and weights, computed once per workgroup
  __shared__ double nsh[EST_CHUNK], wsh[EST_CHUNK];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = blockIdx.y, m = blockIdx.z;
  const int nch = gridDim.y;
  const double mx = fstat[(size_t)m * FREC + 0];
  const bool deg = fstat[(size_t)m * FREC + 3] != 0.0;
  const int i0 = ch * EST_CHUNK, i1 = min(N, i0 + EST_CHUNK);
  for (int k = threadIdx.x; k < i1 - i0; k += blockDim.x) {
    nsh[k] = (double)cnt[(size_t)m * N + i0 + k];
    wsh[k] = deg ? 1.0 : exp((double)lw[(size_t)m * N + i0 + k] - mx);
  }
  __syncthreads();
  if (g >= dx4) return;
  double pv[4] = {0, 0, 0, 0}, wv[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const float4 x = ld_stream(Xb + ((size_t)m * N + i) * dx4 + g);
    const double n = nsh[i - i0], w = wsh[i - i0];
    pv[0] += n * x.x; pv[1] += n * x.y; pv[2] += n * x.z; pv[3] += n * x.w;
    wv[0] += w * x.x; wv[1] += w * x.y; wv[2] += w * x.z; wv[3] += w * x.w;
  }
  double *o = part + (((size_t)m * nch + ch) * 2) * (size_t)dx4 * 4;
  for (int l = 0; l < 4; ++l) {
    o[(size_t)g * 4 + l] = pv[l];
    o[(size_t)dx4 * 4 + (size_t)g * 4 + l] = wv[l];
  }
}

// Filter means from the chunk partials: a workgroup per (64 state elements,
// filter), its four waves each summing every fourth chunk of the filter's
// (ch = slice, slice + 4, ...: one coalesced 512-byte row per wave and
// chunk), the four slices added in LDS in slice order.
constexpr int FOLD_COLS = 64, FOLD_SLICES = GB / FOLD_COLS;
__global__ void __launch_bounds__(GB)
k_grid_filter_fold(int N, int dx, int nch, const double *__restrict__ part,
                   const double *__restrict__ fstat, double *__restrict__ fmean,
                   double *__restrict__ fmeanw) {
  __shared__ double sa[FOLD_SLICES][FOLD_COLS], sb[FOLD_SLICES][FOLD_COLS];
  const int cl = threadIdx.x % FOLD_COLS, sl = threadIdx.x / FOLD_COLS;
  const int c = blockIdx.x * FOLD_COLS + cl, m = blockIdx.y;
  double a = 0.0, b = 0.0;
  if (c < dx) {
#pragma unroll 4
    for (int ch = sl; ch < nch; ch += FOLD_SLICES) {
      const double *o = part + (((size_t)m * nch + ch) * 2) * (size_t)dx;
      a += o[c];
      b += o[(size_t)dx + c];
    }
  }
  sa[sl][cl] = a;
  sb[sl][cl] = b;
  __syncthreads();
  if (sl != 0 || c >= dx) return;
#pragma unroll
  for (int q = 1; q < FOLD_SLICES; ++q) {
    a += sa[q][cl];
    b += sb[q][cl];
  }
  const double W = fstat[(size_t)m * FREC + 1];
  // a filter that kept its particles (ESS schedule) reports the weighted mean
  const bool kept = fstat[(size_t)m * FREC + FREC_KEPT] != 0.0;
  fmean[(size_t)m * dx + c] = kept ? b / W : a / (double)N;
  fmeanw[(size_t)m * dx + c] = b / W;
}

// Ensemble means: a workgroup per 64 state elements, its four waves each
// summing every fourth filter's means (m = slice, slice + 4, ...), the four
// slices added in LDS in slice order.
__global__ void __launch_bounds__(GB)
k_grid_ensemble_fold(int M, int dx, const double *__restrict__ fmean,
                     const double *__restrict__ fmeanw, double *__restrict__ emean) {
  __shared__ double sa[FOLD_SLICES][FOLD_COLS], sb[FOLD_SLICES][FOLD_COLS];
  const int cl = threadIdx.x % FOLD_COLS, sl = threadIdx.x / FOLD_COLS;
  const int c = blockIdx.x * FOLD_COLS + cl;
  double a = 0.0, b = 0.0;
  if (c < dx) {
#pragma unroll 4
    for (int m = sl; m < M; m += FOLD_SLICES) {
      a += fmean[(size_t)m * dx + c];
      b += fmeanw[(size_t)m * dx + c];
    }
  }
  sa[sl][cl] = a;
  sb[sl][cl] = b;
  __syncthreads();
  if (sl != 0 || c >= dx) return;
#pragma unroll
  for (int q = 1; q < FOLD_SLICES; ++q) {
    a += sa[q][cl];
    b += sb[q][cl];
  }
  emean[c] = a / (double)M;
  emean[dx + c] = b / (double)M;
}

// The estimator kernels above over tables of ensembles (fused path): the
// partials of job {ensemble, filter, chunk} from the buffer `out`, the fold
// of job {ensemble, filter}, the ensemble fold of the listed ensembles.
__global__ void __launch_bounds__(GB)
k_grid_estimate_part_b(const int4 *__restrict__ jobs, const FusedEns *__restrict__ ens, int out,
                       int dx4) {
  // the chunk's offspring counts and weights, computed once per workgroup
  __shared__ double nsh[EST_CHUNK], wsh[EST_CHUNK];
  const int4 jb = jobs[blockIdx.x];
  const FusedEns &E = ens[jb.x];
  const int g = blockIdx.y * GB + threadIdx.x;
  const int m = jb.y, ch = jb.z, N = E.N, nch = E.nch;
  // (pointers from the ensemble table: global-address-space accesses)
  const gmem<f4v> *Xb = gptr((const f4v *)(out ? E.X1 : E.X0));
  const double mx = gptr(E.fstat)[(size_t)m * FREC + 0];
  const bool deg = gptr(E.fstat)[(size_t)m * FREC + 3] != 0.0;
  const int i0 = ch * EST_CHUNK, i1 = min(N, i0 + EST_CHUNK);
  for (int k = threadIdx.x; k < i1 - i0; k += GB) {
    nsh[k] = (double)gptr(E.cnt)[(size_t)m * N + i0 + k];
    wsh[k] = deg ? 1.0 : exp((double)gptr(E.lw)[(size_t)m * N + i0 + k] - mx);
  }
  __syncthreads();
  if (g >= dx4) return;
  double pv[4] = {0, 0, 0, 0}, wv[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const f4v x = __builtin_nontemporal_load(Xb + ((size_t)m * N + i) * dx4 + g);
    const double n = nsh[i - i0], w = wsh[i - i0];
    pv[0] += n * x.x; pv[1] += n * x.y; pv[2] += n * x.z; pv[3] += n * x.w;
    wv[0] += w * x.x; wv[1] += w * x.y; wv[2] += w * x.z; wv[3] += w * x.w;
  }
  gmem<double> *o = gptr(E.gpart + (((size_t)m * nch + ch) * 2) * (size_t)dx4 * 4);
  for (int l = 0; l < 4; ++l) {
    o[(size_t)g * 4 + l] = pv[l];
    o[(size_t)dx4 * 4 + (size_t)g * 4 + l] = wv[l];
  }
}

__global__ void __launch_bounds__(GB)
k_grid_filter_fold_b(const int4 *__restrict__ jobs, const FusedEns *__restrict__ ens, int dx) {
  const int4 jb = jobs[blockIdx.x];
  const FusedEns &E = ens[jb.x];
  const int c = blockIdx.y * GB + threadIdx.x, m = jb.y, nch = E.nch;
  if (c >= dx) return;
  double a = 0.0, b = 0.0;
  // (unrolled: the loads of several terms issue before their in-order sums)
#pragma unroll 8
  for (int ch = 0; ch < nch; ++ch) {
    const gmem<double> *o = gptr(E.gpart + (((size_t)m * nch + ch) * 2) * (size_t)dx);
    a += o[c];
    b += o[(size_t)dx + c];
  }
  const double W = gptr(E.fstat)[(size_t)m * FREC + 1];
  // a filter that kept its particles (ESS schedule) reports the weighted mean
  const bool kept = gptr(E.fstat)[(size_t)m * FREC + FREC_KEPT] != 0.0;
  gptr(E.fmean)[(size_t)m * dx + c] = kept ? b / W : a / (double)E.N;
  gptr(E.fmeanw)[(size_t)m * dx + c] = b / W;
}

__global__ void __launch_bounds__(GB)
k_grid_ensemble_fold_b(const int *__restrict__ gens, const FusedEns *__restrict__ ens, int dx) {
  const FusedEns &E = ens[gens[blockIdx.x]];
  const int c = blockIdx.y * GB + threadIdx.x;
  if (c >= dx) return;
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (int m = 0; m < E.M; ++m) {
    a += gptr(E.fmean)[(size_t)m * dx + c];
    b += gptr(E.fmeanw)[(size_t)m * dx + c];
  }
  gptr(E.emean)[c] = a / (double)E.M;
  gptr(E.emean)[dx + c] = b / (double)E.M;
}

// Truth path on the truth stream: one workgroup, T intervals of S steps.
template <int SPT>
__global__ void __launch_bounds__(1024)
k_grid_simulate(ModelDev md, Key key, int T, float *__restrict__ xtrue, float *__restrict__ y) {
  extern __shared__ float vs[];
  const int J = md.J, nn = J * J, slots = nn / 4, dx = 2 * nn;
  Nbr4 nb[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) nb[q] = neighbours(J, min((int)(threadIdx.x + q * blockDim.x), slots - 1));
  Slot4 S[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int s = threadIdx.x + q * blockDim.x;
    if (s < slots) {
      float z[4], v[4], w[4];
      // state index of v at node 4s+l is 4s+l, of w is nn + 4s+l
      normals4(philox(0u, TRUTH_STREAM, 0u, (P_TRUTH_INIT << 24) | (uint32_t)s, key), z);
      for (int l = 0; l < 4; ++l) v[l] = md.prior_mean[4 * s + l] + md.prior_sd[4 * s + l] * z[l];
      normals4(philox(0u, TRUTH_STREAM, 0u, (P_TRUTH_INIT << 24) | (uint32_t)(slots + s), key), z);
      for (int l = 0; l < 4; ++l)
        w[l] = md.prior_mean[nn + 4 * s + l] + md.prior_sd[nn + 4 * s + l] * z[l];
      S[q].start(make_float4(v[0], v[1], v[2], v[3]), make_float4(w[0], w[1], w[2], w[3]));
      *(float4 *)(vs + 4 * s) = S[q].v;
      ((float4 *)xtrue)[s] = S[q].v;
      ((float4 *)xtrue)[slots + s] = S[q].w;
    }
  }
  __syncthreads();
  for (int t = 1; t <= T; ++t) {
    for (int st = 0; st < md.S; ++st) {
      const uint32_t n = (uint32_t)((t - 1) * md.S + st);
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int s = threadIdx.x + q * blockDim.x;
        if (s < slots)
          grid_euler<EULER_OFFSET>(md, key, P_TRUTH_NOISE, 0u, TRUTH_STREAM, n, s, nb[q], vs, S[q]);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int s = threadIdx.x + q * blockDim.x;
        if (s < slots) *(float4 *)(vs + 4 * s) = S[q].v;
      }
      __syncthreads();
    }
    float4 *xt = (float4 *)(xtrue + (size_t)t * dx);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int s = threadIdx.x + q * blockDim.x;
      if (s < slots) {
        xt[s] = S[q].v;
        xt[slots + s] = S[q].w;
        S[q].start(S[q].v, S[q].w);  // the next interval's offsets from here
      }
    }
    for (int k4 = threadIdx.x; 4 * k4 < md.dy; k4 += GB) {
      float z[4];
      normals4(philox(0u, TRUTH_STREAM, (uint32_t)t, (P_OBS_NOISE << 24) | (uint32_t)k4, key), z);
      for (int l = 0; l < 4 && 4 * k4 + l < md.dy; ++l)
        y[(size_t)(t - 1) * md.dy + 4 * k4 + l] = vs[md.obs_idx[4 * k4 + l]] + md.obs_sd * z[l];
    }
    __syncthreads();
  }
}

size_t grid_lds(const ModelDev &md) { return sizeof(float) * ((size_t)md.J * md.J + 16); }

// k_grid_steps: threads and LDS for ppb particles per workgroup
int steps_threads(int J, int ppb) { return 64 * ((ppb * J * J / 4 + 63) / 64); }
size_t steps_lds(int J, int ppb) { return sizeof(float) * (size_t)ppb * J * J; }

}  // namespace

namespace {
// slots per thread and threads per workgroup of the stepping kernels
void grid_shape(const ModelDev &md, int *spt, int *threads) {
  const int slots = md.J * md.J / 4;
  int k = 1;
  while (k < 4 && 64 * ((slots + 64 * k - 1) / (64 * k)) > 1024) k <<= 1;
  *spt = k;
  *threads = 64 * ((slots + 64 * k - 1) / (64 * k));
}
}  // namespace

// Particles per workgroup of k_grid_steps.  The kernel is VALU-bound, so
// the criterion is the share of useful lanes among the wavefront lanes it
// issues (ppb * slots / threads), among the shapes that keep at least 3
// workgroups and 16 wavefronts resident per CU (the other workgroups' waves
// cover each workgroup's two barriers per Euler step; measured: for J = 40,
// one particle in 4 resident workgroups of 7 waves beats two in 2 of 13).
// Cached per J (the launch and the table padding must agree).
namespace {
template <bool ROW4>
hipError_t steps_occupancy(int *per_cu, int J, int ppb) {
  return ppb == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_grid_steps<ROW4>, steps_threads(J, 1), steps_lds(J, 1))
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_grid_steps_multi<ROW4>, steps_threads(J, ppb), steps_lds(J, ppb));
}
int steps_blocks_per_cu(int J, int ppb) {
  int per_cu = 0;
  const hipError_t e = J % 4 == 0 ? steps_occupancy<true>(&per_cu, J, ppb)
                                  : steps_occupancy<false>(&per_cu, J, ppb);
  return e == hipSuccess ? per_cu : 0;
}
}  // namespace

int grid_steps_ppb(int J) {
  static std::atomic<int> cache[65];
  if (J < 2 || J > 64) return 1;
  const int c = cache[J].load(std::memory_order_relaxed);
  if (c > 0) return c;
  const int slots = J * J / 4;
  int best = 1, best_waves = 0;
  double best_fill = -1.0;
  bool best_ok = false;
  for (int k = 1; k <= 8 && k * slots <= 1024; ++k) {
    const int threads = steps_threads(J, k), blocks = steps_blocks_per_cu(J, k);
    const int waves = blocks * threads / 64;
    const double fill = (double)(k * slots) / threads;
    const bool ok = blocks >= 3 && waves >= 16;
    if ((ok && !best_ok) || (ok == best_ok && (ok ? fill > best_fill + 1e-9 : waves > best_waves))) {
      best = k;
      best_fill = fill;
      best_waves = waves;
      best_ok = ok;
    }
  }
  cache[J].store(best, std::memory_order_relaxed);
  return best;
}

int grid_resident_blocks_j(int J) {
  const int ppb = grid_steps_ppb(J);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1024;
  return std::max(1, steps_blocks_per_cu(J, ppb)) * prop.multiProcessorCount;
}

// resident workgroups of the streaming one-step kernel
int grid_resident_blocks(const ModelDev &md) {
  int dev = 0, per_cu = 0, spt, threads;
  grid_shape(md, &spt, &threads);
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1024;
  const size_t lds = grid_lds(md);
  hipError_t e = spt == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_grid_stream_step<1>, threads, lds)
               : spt == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_grid_stream_step<2>, threads, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_grid_stream_step<4>, threads, lds);
  if (e != hipSuccess) return 1024;
  return std::max(1, per_cu) * prop.multiProcessorCount;
}

hipError_t launch_grid_pilot(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s) {
  const size_t lds = sizeof(float) * (3 * (size_t)J * J + PILOT_THREADS / 64);
  k_grid_pilot<<<(unsigned)((size_t)M * N), PILOT_THREADS, lds, s>>>(d_ens, e, iv, parity, pending);
  return hipGetLastError();
}

hipError_t launch_grid_init(const EnsDev &e, float *X, hipStream_t s) {
  k_grid_init<<<e.M * e.N, GB, 0, s>>>(e.md, e.key, e.N, X);
  return hipGetLastError();
}

hipError_t launch_grid_steps_batched(int J, const int4 *d_ptab, int n_p, const FusedEns *d_ens,
                                     IvArg iv, int parity, int pending, int blocks, hipStream_t s) {
  if (n_p <= 0) return hipSuccess;
  const int ppb = grid_steps_ppb(J);
  if (n_p % ppb != 0) return hipErrorInvalidValue;  // the table is padded per ensemble
  const int g = std::max(1, std::min(blocks, n_p / ppb));
  const int th = steps_threads(J, ppb);
  const size_t lds = steps_lds(J, ppb);
  const bool row4 = J % 4 == 0;
  if (ppb == 1 && row4)
    k_grid_steps<true><<<g, th, lds, s>>>(d_ptab, n_p, d_ens, iv, parity, pending, J);
  else if (ppb == 1)
    k_grid_steps<false><<<g, th, lds, s>>>(d_ptab, n_p, d_ens, iv, parity, pending, J);
  else if (row4)
    k_grid_steps_multi<true><<<g, th, lds, s>>>(d_ptab, n_p, d_ens, iv, parity, pending, J, ppb);
  else
    k_grid_steps_multi<false><<<g, th, lds, s>>>(d_ptab, n_p, d_ens, iv, parity, pending, J, ppb);
  return hipGetLastError();
}

hipError_t launch_grid_estimate_batched(int J, const int4 *d_part_jobs, int n_part,
                                        const int4 *d_fold_jobs, int n_fold, const int *d_gens,
                                        int n_gens, const FusedEns *d_ens, int out, hipStream_t s) {
  if (n_gens <= 0) return hipSuccess;
  const int dx = 2 * J * J, dx4 = dx / 4;
  k_grid_estimate_part_b<<<dim3(n_part, (dx4 + GB - 1) / GB), GB, 0, s>>>(d_part_jobs, d_ens, out,
                                                                          dx4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_grid_filter_fold_b<<<dim3(n_fold, (dx + GB - 1) / GB), GB, 0, s>>>(d_fold_jobs, d_ens, dx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_grid_ensemble_fold_b<<<dim3(n_gens, (dx + GB - 1) / GB), GB, 0, s>>>(d_gens, d_ens, dx);
  return hipGetLastError();
}

hipError_t launch_grid_stream_step(const EnsDev &e, int n, const float *Xin, const int32_t *anc,
                                   float *Xout, float *lw, const float *y, int blocks,
                                   hipStream_t s) {
  int spt, threads;
  grid_shape(e.md, &spt, &threads);
  const int g = std::min(blocks, e.M * e.N);
  const size_t lds = grid_lds(e.md);
  if (spt == 1)
    k_grid_stream_step<1><<<g, threads, lds, s>>>(e.md, e.key, e.M, e.N, n, Xin, anc, Xout, lw, y);
  else if (spt == 2)
    k_grid_stream_step<2><<<g, threads, lds, s>>>(e.md, e.key, e.M, e.N, n, Xin, anc, Xout, lw, y);
  else
    k_grid_stream_step<4><<<g, threads, lds, s>>>(e.md, e.key, e.M, e.N, n, Xin, anc, Xout, lw, y);
  return hipGetLastError();
}

hipError_t launch_grid_loglik(const EnsDev &e, const float *X, const float *y, hipStream_t s) {
  const int total = e.M * e.N;
  k_grid_loglik<<<(total + GB - 1) / GB, GB, 0, s>>>(e.md, e.M, e.N, X, y, e.lw);
  return hipGetLastError();
}

hipError_t launch_grid_gather(const EnsDev &e, const float *Xin, float *Xout, hipStream_t s) {
  const int dx4 = e.md.dx / 4;
  k_grid_gather<<<e.M * e.N, GB, 0, s>>>(e.N, dx4, e.A, (const float4 *)Xin, (float4 *)Xout);
  return hipGetLastError();
}

int grid_est_chunks(int N) { return (N + EST_CHUNK - 1) / EST_CHUNK; }

hipError_t launch_grid_estimate(const EnsDev &e, const float *Xb, const int32_t *cnt,
                                double *part, hipStream_t s) {
  const int dx4 = e.md.dx / 4, nch = grid_est_chunks(e.N);
  // the state's float4 groups split evenly over the fewest workgroups of at
  // most GB threads (e.g. 519 groups: 3 x 192 threads rather than 3 x 256)
  const int ngr = (dx4 + GB - 1) / GB;
  const int th = std::min(GB, 64 * (((dx4 + ngr - 1) / ngr + 63) / 64));
  dim3 g((unsigned)((dx4 + th - 1) / th), (unsigned)nch, (unsigned)e.M);
  k_grid_estimate_part<<<g, th, 0, s>>>(e.N, dx4, (const float4 *)Xb, cnt, e.lw, e.fstat, part);
  const dim3 gf((unsigned)((e.md.dx + FOLD_COLS - 1) / FOLD_COLS), (unsigned)e.M);
  k_grid_filter_fold<<<gf, GB, 0, s>>>(e.N, e.md.dx, nch, part, e.fstat, e.fmean, e.fmeanw);
  k_grid_ensemble_fold<<<(e.md.dx + FOLD_COLS - 1) / FOLD_COLS, GB, 0, s>>>(e.M, e.md.dx, e.fmean,
                                                                             e.fmeanw, e.emean);
  return hipGetLastError();
}

hipError_t launch_grid_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                                hipStream_t s) {
  int spt, threads;
  grid_shape(e.md, &spt, &threads);
  const size_t lds = grid_lds(e.md);
  if (spt == 1)
    k_grid_simulate<1><<<1, threads, lds, s>>>(e.md, make_key(seed), T, xtrue, y);
  else if (spt == 2)
    k_grid_simulate<2><<<1, threads, lds, s>>>(e.md, make_key(seed), T, xtrue, y);
  else
    k_grid_simulate<4><<<1, threads, lds, s>>>(e.md, make_key(seed), T, xtrue, y);
  return hipGetLastError();
}

}  // namespace pfk
