// pf_device.h -- device primitives shared by the gfx950 kernels: the
// Philox4x32-10 counter-based generator, the uniform and Box-Muller maps,
// wave64 / workgroup reductions and scans, and the device-side model record.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// ---------------------------------------------------------------------------
// Global-memory views of pointers the compiler cannot prove global (loaded
// from device-side tables): accesses through them compile to global_* rather
// than flat_* instructions, which would also hold the LDS wait counter.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ const gmem<T> *gptr(const T *p) {
  return (const gmem<T> *)p;
}
template <class T>
__device__ __forceinline__ gmem<T> *gptr(T *p) {
  return (gmem<T> *)p;
}

// Order-preserving 32-bit keys of floats, for a maximum taken with integer
// atomics: a non-negative float gets its sign bit set, a negative one all its
// bits flipped, so the unsigned order of keys is the order of the values
// (-inf -> 0x007FFFFF).  Key 0 stands for "no value yet" (it is the key of no
// float that is not a NaN) and reads back as -inf.
__device__ __forceinline__ uint32_t ord_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  if (k == 0u) return -INFINITY;
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// ---------------------------------------------------------------------------
// Random numbers.  Philox4x32-10 (Salmon et al., SC'11): per round two 32x32
// -> 64-bit products of counter words 0 and 2 with the published multipliers,
// the Weyl key schedule, ten rounds.  The counter layout that every kernel
// uses: (c0, c1, c2, purpose << 24 | sub-block), key = (seed_lo, seed_hi ^
// 0x14078071).
enum : uint32_t {
  P_INIT = 1, P_PROP = 2, P_RESAMPLE = 3, P_TRUTH_INIT = 4,
  P_TRUTH_NOISE = 5, P_OBS_NOISE = 6, P_TRAIN = 7
};
constexpr uint32_t TRUTH_STREAM = 0xFFFFFFFFu;

struct Key {
  uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed) {
  return Key{(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x14078071u};
}

// Three-way XOR: one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c) instead of
// two v_xor_b32.  Worth it only when at most one operand is uniform across
// the wavefront (otherwise the plain form computes the uniform part on the
// scalar unit and the bitop3 would need a VGPR copy).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10.  N0_FROM / N2_FROM: the first round whose new word 0 / 2 is
// taken with xor3, i.e. from which both counter words entering it vary
// across lanes.  With one per-lane counter word at the start every word is
// per-lane after four rounds (the default); a per-lane c0 (particle or
// element index, uniform c1..c3) gets there for word 0 in round 2 and for
// word 2 in round 3.
template <int N0_FROM = 4, int N2_FROM = 4>
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = r >= N0_FROM ? xor3((uint32_t)(p1 >> 32), c1, k0)
                                     : (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = r >= N2_FROM ? xor3((uint32_t)(p0 >> 32), c3, k1)
                                     : (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// u = (2 (x >> 9) + 1) 2^-24 in (0, 1): the integer has at most 24
// significant bits, so the float is exact.  Formed without an
// integer-to-float conversion (a half-rate instruction): the bit pattern
// 0x3F800000 | (x >> 9) -- one v_alignbit_b32, the low word of the 64-bit
// pair (0x7F : x) shifted right by 9 -- is the float 1 + (x >> 9) 2^-23 in
// [1, 2), and subtracting the float 1 - 2^-24 leaves exactly
// (2 (x >> 9) + 1) 2^-24, which is representable, so the subtraction does
// not round.
__device__ __forceinline__ float u01f(uint32_t x) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9)) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double u01d(uint32_t x) {
  return (double)((x >> 9) * 2u + 1u) * 0x1p-24;
}

// Box-Muller pair: r = sqrt(-2 ln u0), (r cos 2 pi u1, r sin 2 pi u1).  The
// hardware log2 and sine/cosine take the argument in revolutions, which is
// exactly what u1 is.
__device__ __forceinline__ float2 box_muller(uint32_t a, uint32_t b) {
  const float u0 = u01f(a);
  const float u1 = u01f(b);
  // u0 >= 2^-24, so the argument of the square root is a normal float in
  // (0, 33.3]: the raw hardware square root needs no denormal scaling.
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
  return make_float2(r * __builtin_amdgcn_cosf(u1), r * __builtin_amdgcn_sinf(u1));
}

__device__ __forceinline__ void normals4(uint4 w, float z[4]) {
  const float2 a = box_muller(w.x, w.y);
  const float2 b = box_muller(w.z, w.w);
  z[0] = a.x; z[1] = a.y; z[2] = b.x; z[3] = b.y;
}

// ---------------------------------------------------------------------------
// Model record handed to kernels by value.
struct ModelDev {
  int32_t kind;      // 0 OU, 1 Lorenz 63, 2 FH-N, 3 the paper's FH-N network
  int32_t dx, J, S, dy;
  float h;
  float p0, p1, p2, p3;   // model parameters
  float sq0, sq1;         // noise_sd * sqrt(h) per variable class
  float inv2var;          // 1 / (2 obs_var)
  float obs_sd;           // sqrt(obs_var)
  const int32_t *obs_idx; // [dy]
  const float *prior_mean, *prior_sd; // [dx]
  // the paper's network (kind 3): recovery constant, stimulus amplitude,
  // band (lo, hi) of the stimulus region, Bernoulli parameter, stimulus
  // duration l0 (steps), forcing period and pulse width (steps)
  float stim_b2, stim_amp, stim_lo, stim_hi;
  double stim_eps;
  int32_t stim_l0, force_period, force_width;
};

// One Euler-Maruyama step of one FH-N node from its v (c), w, the 5-point
// Laplacian of v and the two normals: drift v(v-a)(1-v) - w + D lap,
// eps (v - gam w), plus (DRIFT) the proposal's drift corrections uv, uw; the
// increments are added with compensated (Kahan) sums whose running
// corrections cv, cw live with the caller.
template <bool DRIFT>
__device__ __forceinline__ void fhn_node_step(const ModelDev &md, float c, float w, float lap,
                                              float zv, float zw, float uv, float uw, float &v_new,
                                              float &w_new, float &cv, float &cw) {
  float fv = c * (c - md.p0) * (1.f - c) - w + md.p1 * lap;
  float fw = md.p2 * (c - md.p3 * w);
  if (DRIFT) {
    fv += uv;
    fw += uw;
  }
  const float iv = fmaf(md.h, fv, md.sq0 * zv) - cv;
  const float nv = c + iv;
  cv = (nv - c) - iv;
  v_new = nv;
  const float iw = fmaf(md.h, fw, md.sq1 * zw) - cw;
  const float nw = w + iw;
  cw = (nw - w) - iw;
  w_new = nw;
}

// The same step with the increments summed in an FP32 offset from the
// interval's start state (v0, w0): dv, dw hold the sums so far, and the new
// state is v0 + dv, w0 + dw -- rounded once from the start state, like the
// compensated form, for four arithmetic instructions per variable instead
// of six.
template <bool DRIFT>
__device__ __forceinline__ void fhn_node_step_off(const ModelDev &md, float c, float w, float lap,
                                                  float zv, float zw, float uv, float uw, float v0,
                                                  float w0, float &v_new, float &w_new, float &dv,
                                                  float &dw) {
  float fv = c * (c - md.p0) * (1.f - c) - w + md.p1 * lap;
  float fw = md.p2 * (c - md.p3 * w);
  if (DRIFT) {
    fv += uv;
    fw += uw;
  }
  dv += fmaf(md.h, fv, md.sq0 * zv);
  v_new = v0 + dv;
  dw += fmaf(md.h, fw, md.sq1 * zw);
  w_new = w0 + dw;
}

// ---------------------------------------------------------------------------
// Wave64 and workgroup reductions / scans.  The wave level uses DPP lane
// moves (row shifts within 16-lane rows, then the row broadcasts of lanes 15
// and 31): a Hillis-Steele inclusive scan in six VALU steps, without the LDS
// crossbar that a generic shuffle goes through.  Called by every lane of the
// wave (full EXEC).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v, int identity) {
  // lanes whose source is outside the pattern, or whose row is masked off,
  // receive the identity
  return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {  // identity +0.0
  const int lo = dpp_i32<CTRL, ROWS>(__double2loint(v), 0);
  const int hi = dpp_i32<CTRL, ROWS>(__double2hiint(v), 0);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118, DPP_WAVE_SHR1 = 0x138, DPP_ROW_BCAST15 = 0x142,
              DPP_ROW_BCAST31 = 0x143;

__device__ __forceinline__ float wave_max(float v) {
  const int id = __float_as_int(-INFINITY);
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_SHR1, 0xf>(__float_as_int(v), id)));
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_SHR2, 0xf>(__float_as_int(v), id)));
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_SHR4, 0xf>(__float_as_int(v), id)));
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_SHR8, 0xf>(__float_as_int(v), id)));
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_BCAST15, 0xa>(__float_as_int(v), id)));
  v = fmaxf(v, __int_as_float(dpp_i32<DPP_ROW_BCAST31, 0xc>(__float_as_int(v), id)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// inclusive scan across the 64 lanes
__device__ __forceinline__ double wave_scan(double v) {
  v += dpp_f64<DPP_ROW_SHR1, 0xf>(v);
  v += dpp_f64<DPP_ROW_SHR2, 0xf>(v);
  v += dpp_f64<DPP_ROW_SHR4, 0xf>(v);
  v += dpp_f64<DPP_ROW_SHR8, 0xf>(v);
  v += dpp_f64<DPP_ROW_BCAST15, 0xa>(v);
  v += dpp_f64<DPP_ROW_BCAST31, 0xc>(v);
  return v;
}
// the wave total (the scan's last lane), in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v = wave_scan(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Workgroup max over blockDim.x threads (multiple of 64, <= 1024).
__device__ __forceinline__ float block_max(float v, float *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < nw; ++i) r = fmaxf(r, sh[i]);
  return r;
}
// Workgroup sum in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}
// Workgroup sums of R values at once (fixed order); the results are valid in
// thread 0 only (the other threads skip the fold).  sh holds
// R * (blockDim.x / 64) doubles.
template <int R>
__device__ __forceinline__ void block_sum_multi_t0(double v[R], double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = wave_sum(v[r]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) sh[r * nw + wid] = v[r];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double a = 0.0;
      for (int i = 0; i < nw; ++i) a += sh[r * nw + i];
      v[r] = a;
    }
  }
}

// Workgroup sums of R <= 64 values at once (fixed order, that of
// block_sum_multi_t0); thread r < R returns the sum of value r, so that the
// R final folds run side by side in the lanes of wave 0.  sh holds
// R * (blockDim.x / 64) doubles.
template <int R>
__device__ __forceinline__ double block_sum_multi_lane(double v[R], double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = wave_sum(v[r]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) sh[r * nw + wid] = v[r];
  }
  __syncthreads();
  double a = 0.0;
  if (threadIdx.x < R)
    for (int i = 0; i < nw; ++i) a += sh[threadIdx.x * nw + i];
  return a;
}

// Workgroup exclusive scan; returns the exclusive prefix of this thread and
// the total in *tot.
__device__ __forceinline__ double block_exscan(double v, double *sh, double *tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double inc = wave_scan(v);
  const double exc = dpp_f64<DPP_WAVE_SHR1, 0xf>(inc);  // lane 0 receives 0
  __syncthreads();
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  double off = 0.0, all = 0.0;
  for (int i = 0; i < nw; ++i) {
    if (i < wid) off += sh[i];
    all += sh[i];
  }
  *tot = all;
  return off + exc;
}

// Two workgroup exclusive scans with one pair of barriers (each value's
// arithmetic is that of block_exscan); sh holds 2 * (blockDim.x / 64)
// doubles.
__device__ __forceinline__ void block_exscan2(double v0, double v1, double *sh, double ex[2],
                                              double tot[2]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const double i0 = wave_scan(v0), i1 = wave_scan(v1);
  const double e0 = dpp_f64<DPP_WAVE_SHR1, 0xf>(i0), e1 = dpp_f64<DPP_WAVE_SHR1, 0xf>(i1);
  __syncthreads();
  if (lane == 63) {
    sh[wid] = i0;
    sh[nw + wid] = i1;
  }
  __syncthreads();
  double o0 = 0.0, a0 = 0.0, o1 = 0.0, a1 = 0.0;
  for (int i = 0; i < nw; ++i) {
    if (i < wid) {
      o0 += sh[i];
      o1 += sh[nw + i];
    }
    a0 += sh[i];
    a1 += sh[nw + i];
  }
  ex[0] = o0 + e0;
  ex[1] = o1 + e1;
  tot[0] = a0;
  tot[1] = a1;
}

}  // namespace pfk
