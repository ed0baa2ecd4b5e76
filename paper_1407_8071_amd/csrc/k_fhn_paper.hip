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
// One workgroup of 256 threads advances one particle at a time.  Thread t
// owns the 4Q consecutive nodes 4Q t .. 4Q t + 4Q - 1 (Q = ceil(J*J / 1024)):
// their U, V and stimulus coverage counts stay in registers for the whole
// interval, and only the U plane (read by the neighbours) goes through LDS.
// Per Euler step n:
//   (A) [barrier: the step's input plane is complete] every thread reads the
//       four neighbours of its nodes once, for the coupling sums;
//   (B) one Philox call (particle, filter, n, PROP | sub-block J*J/2), the
//       same in every thread: its first uniform against eps decides the
//       Bernoulli event.  Only when it falls below eps (rare) is the
//       stimulus region formed -- the nodes whose U, or a 4-neighbour's U,
//       lies in the open band (u-, u+) -- and ordered row-major by a wave
//       scan of each thread's count and the wave totals in LDS [barrier];
//       the second uniform picks its floor(u |S|)-th node as the centre
//       (no event when the region is empty), and the thread whose range
//       holds that node publishes it [barrier];
//   (C) the event replaces the ring's entry of step n - l0: every thread
//       updates the coverage counts of its nodes (centre and neighbours of
//       the entering and the leaving event), so that the stimulus of a node
//       is F~ when its count is positive (F~ min{1, sum Q}); the owner of
//       the ring slot writes it after the next barrier, when every wave has
//       read the leaving entry;
//   (D) the Euler step of every node in registers: U' = U + h (p3(U) - V) +
//       h (c sum_nbr U + m F + Psi) + sigma~ sqrt(h) z, V' = V + h (b0 U +
//       b1 V + b2), the normals of node pair p from the FH-N grid layout
//       (call (particle, filter, n, PROP | p): lanes 0, 1 for node 2p, lanes
//       2, 3 for 2p + 1); U' goes into the other plane of the particle's
//       pair, the next step's input.
// One barrier per step when no event is drawn.  A particle has two planes
// (a step's input and output) and a ring, and two particles' sets alternate,
// so that the next particle's plane and ring are written while a slower
// wave still reads this particle's.  The next particle's state is fetched
// into registers while this one steps (its ancestor index one particle
// earlier still); the previous particle's log-likelihood of the observed U
// nodes is summed by wave 0 from its final plane during the next particle's
// first step.
#include "pf_internal.h"

namespace pfk {
namespace {

constexpr int FP_THREADS = 256, FP_WAVES = FP_THREADS / 64;

// streaming access to a particle's state (touched once per interval)
typedef float fp4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(const gmem<float> *p) {
  const fp4v v = __builtin_nontemporal_load((const gmem<fp4v> *)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(gmem<float> *p, float a, float b, float c, float d) {
  const fp4v v = {a, b, c, d};
  __builtin_nontemporal_store(v, (gmem<fp4v> *)p);
}

// per-node bits (fixed for a thread): which grid neighbours exist, whether
// the node is in the forced 2 x 2 corner block, whether it is a node at all
constexpr int NB_UP = 1, NB_DOWN = 2, NB_LEFT = 4, NB_RIGHT = 8, NB_CORNER = 16, NB_VALID = 32;

struct FpLds {
  float *planes;  // 4 U planes [J*J]: the pair 2 q, 2 q + 1 for particles of parity q
  int nn;
  int *rings;     // 2 event rings [32], by particle parity
  int *wsum;      // [FP_WAVES] wave totals of the region count
  int *ev;        // [0]: centre of the step's event; [1 + q]: whether ring q as loaded holds any
  // (offsets, not arrays of pointers: an index into a pointer array that is
  // not a compile-time constant would put the array in scratch memory)
  __device__ float *plane(int k) const { return planes + k * nn; }
  __device__ int *ring(int q) const { return rings + 32 * q; }
};

__device__ __forceinline__ FpLds fp_lds(int nn) {
  extern __shared__ float4 fp_mem4[];
  float *fp_mem = (float *)fp_mem4;
  FpLds L;
  L.planes = fp_mem;
  L.nn = nn;
  L.rings = (int *)(fp_mem + 4 * nn);
  L.wsum = L.rings + 64;
  L.ev = L.wsum + FP_WAVES;
  return L;
}

size_t fhnp_lds_bytes(int J) {
  const size_t nn = (size_t)J * J;
  return sizeof(float) * (4 * nn + 64 + FP_WAVES + 4);
}

// A thread's deferred write of a ring slot (slot -1: none)
struct RingPend {
  int slot, ev;
};

template <int Q>
__device__ __forceinline__ void node_bits(int J, int nb[4 * Q]) {
  const int nn = J * J, k0 = 4 * Q * (int)threadIdx.x;
#pragma unroll
  for (int e = 0; e < 4 * Q; ++e) {
    const int k = k0 + e, i = k / J, j = k - i * J;
    nb[e] = k >= nn ? 0
                    : NB_VALID | (i > 0 ? NB_UP : 0) | (i < J - 1 ? NB_DOWN : 0) |
                          (j > 0 ? NB_LEFT : 0) | (j < J - 1 ? NB_RIGHT : 0) |
                          (i < 2 && j < 2 ? NB_CORNER : 0);
  }
}

// 1 when node k is the centre c or one of its grid neighbours (c < 0: none)
__device__ __forceinline__ int covers(int J, int c, int k) {
  if (c < 0) return 0;
  const int ci = c / J, cj = c - ci * J, i = k / J, j = k - i * J;
  return ((ci == i && abs(cj - j) <= 1) || (cj == j && abs(ci - i) == 1)) ? 1 : 0;
}

// the first normal of a Box-Muller pair alone: r cos 2 pi u1, as box_muller
// computes it
__device__ __forceinline__ float box_muller_cos(uint32_t a, uint32_t b) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01f(a)));
  return r * __builtin_amdgcn_cosf(u01f(b));
}

__device__ __forceinline__ bool in_band(const ModelDev &md, float u) {
  return u > md.stim_lo && u < md.stim_hi;
}

// inclusive scan of small integers across the 64 lanes (DPP row shifts,
// then the row broadcasts)
__device__ __forceinline__ int wave_scan_i32(int v) {
  v += dpp_i32<DPP_ROW_SHR1, 0xf>(v, 0);
  v += dpp_i32<DPP_ROW_SHR2, 0xf>(v, 0);
  v += dpp_i32<DPP_ROW_SHR4, 0xf>(v, 0);
  v += dpp_i32<DPP_ROW_SHR8, 0xf>(v, 0);
  v += dpp_i32<DPP_ROW_BCAST15, 0xa>(v, 0);
  v += dpp_i32<DPP_ROW_BCAST31, 0xc>(v, 0);
  return v;
}

// Coverage counts of a thread's nodes from the ring in LDS (entries
// 0..l0-1, l0 <= 32): all 32 entries in eight broadcast reads, then the
// active ones (usually none) one by one.
template <int Q>
__device__ __forceinline__ void build_cover(int J, int l0, const int nb[4 * Q], const int *ring,
                                            bool any, int cov[4 * Q]) {
  const int k0 = 4 * Q * (int)threadIdx.x;
#pragma unroll
  for (int e = 0; e < 4 * Q; ++e) cov[e] = 0;
  if (!any) return;  // (no entry of the loaded ring holds an event: the usual case)
  unsigned act = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const int4 c = ((const int4 *)ring)[g];
    act |= (c.x >= 0 ? 1u : 0u) << (4 * g);
    act |= (c.y >= 0 ? 1u : 0u) << (4 * g + 1);
    act |= (c.z >= 0 ? 1u : 0u) << (4 * g + 2);
    act |= (c.w >= 0 ? 1u : 0u) << (4 * g + 3);
  }
  if (l0 < 32) act &= (1u << l0) - 1u;
  act = __builtin_amdgcn_readfirstlane(act);
  while (act) {
    const int l = __builtin_ctz(act);
    act &= act - 1u;
    const int c = __builtin_amdgcn_readfirstlane(ring[l]);
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e)
      if (nb[e] & NB_VALID) cov[e] += covers(J, c, k0 + e);
  }
}

// Coupling sums of a thread's nodes (up, down, left, right, those that
// exist, in that order) from the plane pl.  row: the thread's 4Q nodes lie
// in one row (every thread's, or none is a node): the rows above and below
// in 16-byte reads, the outer left and right neighbours in two scalar
// reads, the inner ones from the thread's own registers.
template <int Q>
__device__ __forceinline__ void nbr_sums(int J, int k0, const int nb[4 * Q], const float u[4 * Q],
                                         const float *pl, bool row, float sum[4 * Q]) {
  if (row) {
    if (!(nb[0] & NB_VALID)) {  // (a thread past the last node reads nothing)
#pragma unroll
      for (int e = 0; e < 4 * Q; ++e) sum[e] = 0.f;
      return;
    }
    const bool hu = nb[0] & NB_UP, hd = nb[0] & NB_DOWN;
    const bool hl = nb[0] & NB_LEFT, hr = nb[4 * Q - 1] & NB_RIGHT;
    float up[4 * Q], dn[4 * Q];
#pragma unroll
    for (int g = 0; g < Q; ++g) {
      const float4 a = *(const float4 *)(pl + (hu ? k0 - J : k0) + 4 * g);
      const float4 b = *(const float4 *)(pl + (hd ? k0 + J : k0) + 4 * g);
      up[4 * g] = a.x, up[4 * g + 1] = a.y, up[4 * g + 2] = a.z, up[4 * g + 3] = a.w;
      dn[4 * g] = b.x, dn[4 * g + 1] = b.y, dn[4 * g + 2] = b.z, dn[4 * g + 3] = b.w;
    }
    const float lft = pl[hl ? k0 - 1 : k0], rgt = pl[hr ? k0 + 4 * Q : k0];
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e) {
      float s = 0.f;
      if (hu) s += up[e];
      if (hd) s += dn[e];
      if (e > 0) s += u[e - 1];
      else if (hl) s += lft;
      if (e < 4 * Q - 1) s += u[e + 1];
      else if (hr) s += rgt;
      sum[e] = s;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e) {
      const int k = k0 + e, b = nb[e];
      float s = 0.f;
      if (b & NB_UP) s += pl[k - J];
      if (b & NB_DOWN) s += pl[k + J];
      if (b & NB_LEFT) s += pl[k - 1];
      if (b & NB_RIGHT) s += pl[k + 1];
      sum[e] = s;
    }
  }
}

// Bit e set when node k0 + e is in the stimulus region: its U or a
// 4-neighbour's U lies in the open band (the neighbours read again from pl:
// only on a step that draws an event).
template <int Q>
__device__ __forceinline__ unsigned region_mask(const ModelDev &md, int J, int k0,
                                                const int nb[4 * Q], const float u[4 * Q],
                                                const float *pl, bool row) {
  unsigned rm = 0;
  if (row) {
    if (!(nb[0] & NB_VALID)) return 0u;
    const bool hu = nb[0] & NB_UP, hd = nb[0] & NB_DOWN;
    const bool hl = nb[0] & NB_LEFT, hr = nb[4 * Q - 1] & NB_RIGHT;
    bool ib[4 * Q], bu[4 * Q], bd[4 * Q];
#pragma unroll
    for (int g = 0; g < Q; ++g) {
      const float4 a = *(const float4 *)(pl + (hu ? k0 - J : k0) + 4 * g);
      const float4 b = *(const float4 *)(pl + (hd ? k0 + J : k0) + 4 * g);
      bu[4 * g] = in_band(md, a.x), bu[4 * g + 1] = in_band(md, a.y);
      bu[4 * g + 2] = in_band(md, a.z), bu[4 * g + 3] = in_band(md, a.w);
      bd[4 * g] = in_band(md, b.x), bd[4 * g + 1] = in_band(md, b.y);
      bd[4 * g + 2] = in_band(md, b.z), bd[4 * g + 3] = in_band(md, b.w);
    }
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e) ib[e] = in_band(md, u[e]);
    const bool il = hl && in_band(md, pl[k0 - 1 + (hl ? 0 : 1)]);
    const bool ir = hr && in_band(md, pl[k0 + 4 * Q - (hr ? 0 : 1)]);
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e) {
      const bool r = ib[e] || (hu && bu[e]) || (hd && bd[e]) || (e > 0 ? ib[e - 1] : il) ||
                     (e < 4 * Q - 1 ? ib[e + 1] : ir);
      if ((nb[e] & NB_VALID) && r) rm |= 1u << e;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e) {
      const int k = k0 + e, b = nb[e];
      bool r = in_band(md, u[e]);
      if (b & NB_UP) r |= in_band(md, pl[k - J]);
      if (b & NB_DOWN) r |= in_band(md, pl[k + J]);
      if (b & NB_LEFT) r |= in_band(md, pl[k - 1]);
      if (b & NB_RIGHT) r |= in_band(md, pl[k + 1]);
      if ((b & NB_VALID) && r) rm |= 1u << e;
    }
  }
  return rm;
}

// sum over the 64 lanes (DPP row shifts and broadcasts, as wave_scan_i32),
// in every lane
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += __int_as_float(dpp_i32<DPP_ROW_SHR1, 0xf>(__float_as_int(v), 0));
  v += __int_as_float(dpp_i32<DPP_ROW_SHR2, 0xf>(__float_as_int(v), 0));
  v += __int_as_float(dpp_i32<DPP_ROW_SHR4, 0xf>(__float_as_int(v), 0));
  v += __int_as_float(dpp_i32<DPP_ROW_SHR8, 0xf>(__float_as_int(v), 0));
  v += __int_as_float(dpp_i32<DPP_ROW_BCAST15, 0xa>(__float_as_int(v), 0));
  v += __int_as_float(dpp_i32<DPP_ROW_BCAST31, 0xc>(__float_as_int(v), 0));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// S Euler steps n0 .. n0 + S - 1 of the particle whose nodes this thread
// holds in (u, v, cov), with its input U plane in pa, pb the particle's
// other plane and its ring in LDS; the caller has made pa and the ring
// visible (a barrier).  Step s reads the plane it starts from (pa, pb, pa,
// ...) and writes U' into the other one, so the final U lies in pb for odd
// S and in pa for even S (not yet synchronised).  The ring slot of the last
// step is left in pend (its owner's register pair) for the caller to write.
// PILOT: the auxiliary filter's noise-free continuation -- no new stimulus
// events and no noise; the ring's active stimuli and the forcing act, and
// the ring advances.
template <int Q, bool PILOT>
__device__ __forceinline__ void fhnp_steps(const ModelDev &md, Key key, uint32_t purpose,
                                           uint32_t c0, uint32_t c1, int n0, const int nb[4 * Q],
                                           float u[4 * Q], float v[4 * Q], int cov[4 * Q],
                                           float *pa, float *pb, int *ring, const FpLds &L,
                                           RingPend &pend) {
  const int J = md.J, nn = J * J, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int k0 = 4 * Q * tid;
  const bool row = J % (4 * Q) == 0;
  for (int st = 0; st < md.S; ++st) {
    const uint32_t n = (uint32_t)(n0 + st);
    const float *pin = (st & 1) ? pb : pa;
    float *pout = (st & 1) ? pa : pb;
    if (st > 0) {
      __syncthreads();  // (A) U' of the previous step is complete in pin
      // the previous step's ring entry: every wave has read the one it
      // replaces (with l0 = 1 this step reads that same slot: one more
      // barrier)
      if (pend.slot >= 0) {
        ring[pend.slot] = pend.ev;
        pend.slot = -1;
      }
      if (md.stim_l0 < 2) __syncthreads();
    }
    const int slot = (int)(n % (uint32_t)md.stim_l0);
    const int old = __builtin_amdgcn_readfirstlane(ring[slot]);
    float sum[4 * Q];
    nbr_sums<Q>(J, k0, nb, u, pin, row, sum);
    int ev = -1;
    if (!PILOT) {
      const uint4 r = philox(c0, c1, n, (purpose << 24) | (uint32_t)(nn / 2), key);
      if (u01d(r.x) < md.stim_eps) {  // (the same decision in every thread)
        const unsigned rm = region_mask<Q>(md, J, k0, nb, u, pin, row);
        const int cnt = __builtin_popcount(rm);
        const int inc = wave_scan_i32(cnt);
        if (lane == 63) L.wsum[wid] = inc;
        __syncthreads();
        int off = inc - cnt, total = 0;
#pragma unroll
        for (int w = 0; w < FP_WAVES; ++w) {
          const int ws = L.wsum[w];
          off += w < wid ? ws : 0;
          total += ws;
        }
        total = __builtin_amdgcn_readfirstlane(total);
        int kth = -1;
        if (total > 0) kth = min((int)floor(u01d(r.y) * (double)total), total - 1);
        kth = __builtin_amdgcn_readfirstlane(kth);
        if (kth >= 0) {  // an event
          if (kth >= off && kth < off + cnt) {
            int want = kth - off;
#pragma unroll
            for (int e = 0; e < 4 * Q; ++e)
              if ((rm >> e) & 1u) {
                if (want == 0) L.ev[0] = k0 + e;
                --want;
              }
          }
          __syncthreads();
          ev = __builtin_amdgcn_readfirstlane(L.ev[0]);
        }
      }
    }
    // (C) the ring: ev enters slot n mod l0, the event of step n - l0 leaves
    if (old >= 0 || ev >= 0) {
#pragma unroll
      for (int e = 0; e < 4 * Q; ++e)
        if (nb[e] & NB_VALID) cov[e] += covers(J, ev, k0 + e) - covers(J, old, k0 + e);
      if (tid == (slot >> 2)) {  // the thread that loaded that slot
        pend.slot = slot;
        pend.ev = ev;
      }
    }
    // (D) Euler step of this thread's node pairs
    const bool vnoise = md.sq1 != 0.f;
    const bool forcing = (int)(n % (uint32_t)md.force_period) < md.force_width;
#pragma unroll
    for (int pp = 0; pp < 2 * Q; ++pp) {
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (!PILOT && (nb[2 * pp] & NB_VALID)) {
        const uint4 w = philox(c0, c1, n, (purpose << 24) | (uint32_t)((k0 >> 1) + pp), key);
        if (vnoise) {
          normals4(w, z);
        } else {
          // V without noise: only the U normals (lanes 0 and 2), the same values
          z[0] = box_muller_cos(w.x, w.y);
          z[2] = box_muller_cos(w.z, w.w);
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int e = 2 * pp + q;
        const float uu = u[e], vv = v[e];
        const float psi = cov[e] > 0 ? md.stim_amp : 0.f;
        const float mf = (forcing && (nb[e] & NB_CORNER)) ? md.stim_amp : 0.f;
        const float p3 = md.p0 * uu - uu * uu * uu;
        const float un = (uu + md.h * (p3 - vv)) + md.h * (md.p1 * sum[e] + mf + psi);
        u[e] = fmaf(md.sq0, z[2 * q], un);
        const float vn = vv + md.h * (md.p2 * uu + md.p3 * vv + md.stim_b2);
        v[e] = fmaf(md.sq1, z[2 * q + 1], vn);
      }
    }
#pragma unroll
    for (int g = 0; g < Q; ++g)
      if (nb[4 * g] & NB_VALID)
        *(float4 *)(pout + k0 + 4 * g) =
            make_float4(u[4 * g], u[4 * g + 1], u[4 * g + 2], u[4 * g + 3]);
  }
}

// The previous particle's log-likelihood: the squared residuals of the
// observed U nodes summed by wave 0 alone from that particle's final plane
// (complete: a barrier has passed since its last step), lane 0 writing it.
template <bool PILOT>
struct LikPrev {
  const gmem<float> *y;      // this ensemble's observations (null: none)
  const gmem<int32_t> *obs;  // observed nodes [dy]
  gmem<float> *lw, *lpil;
  const gmem<float> *lwc;
  float inv2var;
  int dy, apf, N;
  const float *plane;  // the previous particle's final plane
  int m, i, src;       // the previous particle and its ancestor
  bool active;
  int o0, o1;          // this lane's first two observations (k = lane, lane + 64): nodes
  float y0, y1;        // and values
  float lpil_src;      // (lane 0, auxiliary filter) the pilot log-likelihood of the ancestor
  __device__ void init_obs() {
    const int k = threadIdx.x & 63;
    o0 = y && k < dy ? obs[k] : 0;
    y0 = y && k < dy ? y[k] : 0.f;
    o1 = y && k + 64 < dy ? obs[k + 64] : 0;
    y1 = y && k + 64 < dy ? y[k + 64] : 0.f;
  }
  __device__ void set(bool on, const float *pl, int pm, int pi, int psrc) {
    active = on;
    plane = pl;
    m = pm;
    i = pi;
    src = psrc;
    // read now, used at the next particle's first step
    if (!PILOT && on && apf && threadIdx.x == 0) lpil_src = lpil[(size_t)pm * N + psrc];
  }
  __device__ void run() {
    if (!active || threadIdx.x >= 64) return;
    const int k = threadIdx.x;
    float acc = 0.f;
    if (k < dy) {
      const float r = y0 - plane[o0];
      acc = r * r;
    }
    if (k + 64 < dy) {
      const float r = y1 - plane[o1];
      acc = fmaf(r, r, acc);
    }
    for (int kk = k + 128; kk < dy; kk += 64) {
      const float r = y[kk] - plane[obs[kk]];
      acc = fmaf(r, r, acc);
    }
    const float a = wave_sum_f32(acc);
    if (k != 0) return;
    float l = -a * inv2var;
    const size_t o = (size_t)m * N + i;
    if (PILOT) {
      // auxiliary filter: the pilot likelihood, kept for the second stage,
      // and the first-stage log-weight lwc + log g(y | mu)
      l = l == l ? l : -INFINITY;
      lpil[o] = l;
      const float lam = l + lwc[o];
      lw[o] = lam == lam ? lam : -INFINITY;
    } else {
      // auxiliary filter: divided by the pilot likelihood of the ancestor
      if (apf) l -= lpil_src;
      lw[o] = l == l ? l : -INFINITY;
    }
  }
};

// Interval t of every particle of fused ensemble e: the state read through
// the ancestors when `pending` (always for an auxiliary filter, whose first
// stage has just drawn them), S steps, state out, log-likelihood when iv
// carries observations.  PILOT: the auxiliary filter's pilot -- S noise-free
// steps without new stimuli, no state out, the pilot likelihood and the
// first-stage log-weight.
template <int Q, bool PILOT>
__global__ void __launch_bounds__(FP_THREADS)
k_fhnp(const FusedEns *__restrict__ ens, int e, IvArg iv, int parity, int pending) {
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t);
  const FusedEns &E = ens[e];
  const ModelDev md = E.md;
  const int J = md.J, nn = J * J, dx = md.dx, N = E.N, MN = E.M * N, G = gridDim.x;
  const int tid = threadIdx.x, k0 = 4 * Q * tid, nr4 = (dx - 2 * nn) / 4;
  const FpLds L = fp_lds(nn);
  const gmem<float> *Xin = gptr(parity ? E.X1 : E.X0);
  gmem<float> *Xout = gptr(parity ? E.X0 : E.X1);
  const gmem<int32_t> *A = gptr(E.A);
  const bool thru = PILOT ? (pending != 0) : (pending || E.apf);
  int nb[4 * Q];
  node_bits<Q>(J, nb);

  // The next particle's state is fetched into registers while this one
  // steps, its ancestor index one particle earlier still.  Both fetches are
  // unconditional (past the end they repeat the last particle, unused), and
  // the index stays raw in a vector register until it is used: the compiler
  // would otherwise move it to a scalar register at once, and waiting for it
  // would also wait for every load issued before it.
  auto anc_raw = [&](int p) {
    p = min(p, MN - 1);
    if (!thru) return p - (p / N) * N;
    // (a fresh opaque zero at every use: kept live across the loop it
    // would be spilled, and its reload would wait for the prefetch)
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    return A[p + vzero];
  };
  auto src_of = [&](int raw) { return min(max(raw, 0), N - 1); };
  float4 fu[Q], fv[Q], fr = make_float4(-1.f, -1.f, -1.f, -1.f);
#pragma unroll
  for (int g = 0; g < Q; ++g) fu[g] = fv[g] = make_float4(0.f, 0.f, 0.f, 0.f);
  auto fetch = [&](int p, int src) {
    const int m = min(p, MN - 1) / N;
    const gmem<float> *x = Xin + ((size_t)m * N + src) * dx;
#pragma unroll
    for (int g = 0; g < Q; ++g)
      if (nb[4 * g] & NB_VALID) {
        fu[g] = ld4(x + k0 + 4 * g);
        fv[g] = ld4(x + nn + k0 + 4 * g);
      }
    if (tid < nr4) fr = ld4(x + 2 * nn + 4 * tid);
  };

  int p = blockIdx.x;
  int src = src_of(anc_raw(p));
  fetch(p, src);
  int raw_nx = anc_raw(p + G);
  LikPrev<PILOT> lik{y ? gptr(y) + E.yoff : nullptr, gptr(md.obs_idx), gptr(E.lw), gptr(E.lpil),
                     gptr((const float *)E.lwc), md.inv2var, md.dy, E.apf, N, L.plane(0),
                     0, 0, 0, false, 0, 0, 0.f, 0.f, 0.f};
  lik.init_obs();
  // A particle's new state is written out at the start of the next
  // iteration, after the prefetched state has been taken from its registers
  // and before the next prefetch is issued: with loads and stores both
  // outstanding, a wait for one kind is a wait for all, and here the only
  // wait for a load comes before the stores and a particle's time after it.
  float u[4 * Q], v[4 * Q];
  int m = 0, i = 0;
  RingPend pend{-1, -1};
  auto store = [&](const int *ring) {
    gmem<float> *x = Xout + ((size_t)m * N + i) * dx;
#pragma unroll
    for (int g = 0; g < Q; ++g)
      if (nb[4 * g] & NB_VALID) {
        st4(x + k0 + 4 * g, u[4 * g], u[4 * g + 1], u[4 * g + 2], u[4 * g + 3]);
        st4(x + nn + k0 + 4 * g, v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
      }
    if (tid < nr4) {
      // (this thread's own ring slots, its deferred write of the last step
      // among them: no other thread writes them)
      float r[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int sl = 4 * tid + c;
        r[c] = sl < md.stim_l0 ? (float)(sl == pend.slot ? pend.ev : ring[sl]) : -1.f;
      }
      st4(x + 2 * nn + 4 * tid, r[0], r[1], r[2], r[3]);
    }
  };
  int par = 0;
  for (; p < MN; p += G) {
    // every load issued in the previous iteration (this particle's state and
    // the next ancestor index) has arrived, issued a particle's time ago; the
    // wait comes before the previous particle's stores, so it never waits
    // for them (s_waitcnt vmcnt(0), the other counters left alone)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    float *pa = L.plane(2 * par), *pb = L.plane(2 * par + 1);
    int *ring = L.ring(par);
    float4 cu[Q], cv[Q];
#pragma unroll
    for (int g = 0; g < Q; ++g) {
      cu[g] = fu[g], cv[g] = fv[g];
      if (nb[4 * g] & NB_VALID) *(float4 *)(pa + k0 + 4 * g) = cu[g];
    }
    const int r0 = (int)fr.x, r1 = (int)fr.y, r2 = (int)fr.z, r3 = (int)fr.w;
    // whether any loaded ring entry holds an event (the loading threads are
    // lanes of wave 0; read after the barrier below)
    const bool mine = tid < nr4 && (r0 >= 0 || r1 >= 0 || r2 >= 0 || r3 >= 0);
    const unsigned long long anyb = __ballot(mine);
    if (tid == 0) L.ev[1 + par] = anyb != 0ull;
    // the previous particle's state out (its ring, of the other parity, is
    // read from LDS before the set of this parity is overwritten two
    // particles on)
    if (!PILOT && p != (int)blockIdx.x) store(L.ring(par ^ 1));
    pend.slot = -1;
    m = p / N;
    i = p - m * N;
    int cov[4 * Q];
#pragma unroll
    for (int g = 0; g < Q; ++g) {
      u[4 * g] = cu[g].x, u[4 * g + 1] = cu[g].y, u[4 * g + 2] = cu[g].z, u[4 * g + 3] = cu[g].w;
      v[4 * g] = cv[g].x, v[4 * g + 1] = cv[g].y, v[4 * g + 2] = cv[g].z, v[4 * g + 3] = cv[g].w;
    }
    if (tid < nr4) {
      ring[4 * tid] = r0;
      ring[4 * tid + 1] = r1;
      ring[4 * tid + 2] = r2;
      ring[4 * tid + 3] = r3;
    }
    const int src_cur = src;
    src = src_of(raw_nx);
    fetch(p + G, src);
    raw_nx = anc_raw(p + 2 * G);
    __syncthreads();  // (A) of step 0: plane and ring complete
    lik.run();        // (wave 0) the previous particle's log-likelihood
    build_cover<Q>(J, md.stim_l0, nb, ring, L.ev[1 + par] != 0, cov);
    fhnp_steps<Q, PILOT>(md, E.key, P_PROP, (uint32_t)i, (uint32_t)m, (t - 1) * md.S, nb, u, v, cov,
                         pa, pb, ring, L, pend);
    lik.set(y != nullptr, (md.S & 1) ? pb : pa, m, i, src_cur);
    par ^= 1;
  }
  if (!PILOT) store(L.ring(par ^ 1));
  if (lik.active) {
    __syncthreads();
    lik.run();
  }
}

// Truth path and observations on the truth stream: one workgroup, T
// intervals of S steps from x_0 ~ tau_0.
template <int Q>
__global__ void __launch_bounds__(FP_THREADS)
k_fhnp_simulate(ModelDev md, Key key, int T, float *__restrict__ xtrue, float *__restrict__ y) {
  const int J = md.J, nn = J * J, dx = md.dx;
  const int tid = threadIdx.x, k0 = 4 * Q * tid, nr4 = (dx - 2 * nn) / 4;
  const FpLds L = fp_lds(nn);
  for (int s = tid; s < dx; s += FP_THREADS) {
    float z[4];
    normals4(philox(0u, TRUTH_STREAM, 0u, (P_TRUTH_INIT << 24) | (uint32_t)(s >> 2), key), z);
    xtrue[s] = md.prior_mean[s] + md.prior_sd[s] * z[s & 3];
  }
  __syncthreads();
  int nb[4 * Q], cov[4 * Q];
  float u[4 * Q], v[4 * Q];
  node_bits<Q>(J, nb);
  float *pa = L.plane(0), *pb = L.plane(1);  // pa: the plane that holds U
  int *ring = L.ring(0);
#pragma unroll
  for (int e = 0; e < 4 * Q; ++e) {
    const bool ok = nb[e] & NB_VALID;
    u[e] = ok ? xtrue[k0 + e] : 0.f;
    v[e] = ok ? xtrue[nn + k0 + e] : 0.f;
    if (ok) pa[k0 + e] = u[e];
  }
  if (tid < nr4)
    for (int c = 0; c < 4; ++c) ring[4 * tid + c] = (int)xtrue[2 * nn + 4 * tid + c];
  __syncthreads();
  build_cover<Q>(J, md.stim_l0, nb, ring, true, cov);
  RingPend pend{-1, -1};
  for (int t = 1; t <= T; ++t) {
    fhnp_steps<Q, false>(md, key, P_TRUTH_NOISE, 0u, TRUTH_STREAM, (t - 1) * md.S, nb, u, v, cov,
                         pa, pb, ring, L, pend);
    if (md.S & 1) {
      float *tmp = pa;
      pa = pb;
      pb = tmp;
    }
    float *x = xtrue + (size_t)t * dx;
#pragma unroll
    for (int e = 0; e < 4 * Q; ++e)
      if (nb[e] & NB_VALID) {
        x[k0 + e] = u[e];
        x[nn + k0 + e] = v[e];
      }
    if (tid < nr4)
      for (int c = 0; c < 4; ++c) {
        const int sl = 4 * tid + c;
        x[2 * nn + sl] = sl < md.stim_l0 ? (float)(sl == pend.slot ? pend.ev : ring[sl]) : -1.f;
      }
    __syncthreads();  // pa holds U at the observation time; every wave has read the last step's ring
    if (pend.slot >= 0) {
      ring[pend.slot] = pend.ev;
      pend.slot = -1;
    }
    if (md.stim_l0 < 2) __syncthreads();  // (the next step reads that same slot)
    for (int k4 = tid; 4 * k4 < md.dy; k4 += FP_THREADS) {
      float z[4];
      normals4(philox(0u, TRUTH_STREAM, (uint32_t)t, (P_OBS_NOISE << 24) | (uint32_t)k4, key), z);
      for (int l = 0; l < 4 && 4 * k4 + l < md.dy; ++l)
        y[(size_t)(t - 1) * md.dy + 4 * k4 + l] = pa[md.obs_idx[4 * k4 + l]] + md.obs_sd * z[l];
    }
    // (the next interval's first step writes pb; pa is written again only
    // after that step's barrier)
  }
}

template <bool PILOT, int Q>
hipError_t launch_q(const FusedEns *d_ens, int e, int MN, int J, IvArg iv, int parity, int pending,
                    hipStream_t s) {
  int per_cu = 0, dev = 0, cus = 256;
  const size_t lds = fhnp_lds_bytes(J);
  // (J = 64: four 16 KB planes, past the default 64 KB of dynamic LDS)
  if (lds > 65536) {
    const hipError_t a = hipFuncSetAttribute((const void *)k_fhnp<Q, PILOT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (a != hipSuccess) return a;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fhnp<Q, PILOT>,
                                                   FP_THREADS, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int blocks = std::min(MN, per_cu * cus);
  k_fhnp<Q, PILOT><<<blocks, FP_THREADS, lds, s>>>(d_ens, e, iv, parity, pending);
  return hipGetLastError();
}

// nodes per thread / 4 on a J x J grid (J even, at most 64)
int fhnp_q(int J) { return (J * J + 4 * FP_THREADS - 1) / (4 * FP_THREADS); }

template <bool PILOT>
hipError_t launch_any(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv, int parity,
                      int pending, hipStream_t s) {
  if (M * N <= 0) return hipSuccess;
  switch (fhnp_q(J)) {
    case 1: return launch_q<PILOT, 1>(d_ens, e, M * N, J, iv, parity, pending, s);
    case 2: return launch_q<PILOT, 2>(d_ens, e, M * N, J, iv, parity, pending, s);
    case 3: return launch_q<PILOT, 3>(d_ens, e, M * N, J, iv, parity, pending, s);
    case 4: return launch_q<PILOT, 4>(d_ens, e, M * N, J, iv, parity, pending, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fhnp_steps(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s) {
  return launch_any<false>(d_ens, e, M, N, J, iv, parity, pending, s);
}

hipError_t launch_fhnp_pilot(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s) {
  return launch_any<true>(d_ens, e, M, N, J, iv, parity, pending, s);
}

hipError_t launch_fhnp_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                                hipStream_t s) {
  const size_t lds = fhnp_lds_bytes(e.md.J);
  const Key key = make_key(seed);
  if (lds > 65536) {
    const void *f = nullptr;
    switch (fhnp_q(e.md.J)) {
      case 3: f = (const void *)k_fhnp_simulate<3>; break;
      case 4: f = (const void *)k_fhnp_simulate<4>; break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t a = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (a != hipSuccess) return a;
  }
  switch (fhnp_q(e.md.J)) {
    case 1: k_fhnp_simulate<1><<<1, FP_THREADS, lds, s>>>(e.md, key, T, xtrue, y); break;
    case 2: k_fhnp_simulate<2><<<1, FP_THREADS, lds, s>>>(e.md, key, T, xtrue, y); break;
    case 3: k_fhnp_simulate<3><<<1, FP_THREADS, lds, s>>>(e.md, key, T, xtrue, y); break;
    case 4: k_fhnp_simulate<4><<<1, FP_THREADS, lds, s>>>(e.md, key, T, xtrue, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pfk
