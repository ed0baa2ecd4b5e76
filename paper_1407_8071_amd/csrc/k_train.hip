// k_train.hip -- training of the learned proposal's network on gfx950.
//
//   k_mlp_grad: minibatch gradient of the mean squared regression loss
//     (1/B) sum_rows |u_theta(x) - target|^2.  Per tile of 16 rows: the
//     forward pass on MFMA (mlp_device.h), the output error, the backward
//     pass through layer 3 on the VALU (out_dim <= 4 terms), through layer 2
//     on MFMA (W2^T against the bfloat16 error of layer 2), and the weight
//     gradients as MFMA products over the 16 rows (v_mfma_f32_16x16x16_bf16,
//     K = rows): the activations and errors go through a per-wave LDS tile
//     [row][unit] so that each lane can read 4 rows of one unit.  The bias of
//     layer 1 is the weight of the constant input, so its gradient comes out
//     of the same product.  Each wave accumulates over its tiles in registers
//     and writes one partial gradient; no atomics.
//   k_grad_reduce_adam: sums the partials over waves in a fixed order (the
//     gradient), optionally followed by the Adam update (Kingma and Ba,
//     Alg. 1) of the FP32 master parameters.
//   k_train_sim: FH-N training paths -- long model runs from tau_0 whose
//     states at the interval ends are the start states, and one-interval
//     trajectories from them with the observation of their end.
//
// Rows of the FH-N regression (trajectory r, step k, node) are drawn per
// Adam step as tiles of 16 consecutive nodes; their features are built from
// the stored trajectory states exactly as the filter builds them, and their
// targets (sd / sqrt(h)) z are regenerated from the trajectory's Philox
// counters.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "mlp_device.h"

namespace pfk {
namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int TR_THREADS = 256;
constexpr int TR_WAVES = TR_THREADS / 64;
constexpr int LROW = 64 + 4;  // bf16 row stride of the per-wave activation tiles
constexpr int XROW = 32 + 4;  // of the input tile
constexpr int DROW = 16 + 4;  // of the output-error tile (16 padded outputs)
// per wave: h1, da2, da1, h2 tiles [16][LROW], input [16][XROW], error [16][DROW]
constexpr int WAVE_LDS = 4 * 16 * LROW + 16 * XROW + 16 * DROW;

// ---- row sources ------------------------------------------------------------
// fill(tile, c, g, F, tgt, ok): features of row c of the tile in this lane's
// K slots (8 g .. 8 g + 7) and, on lanes of group 0, its targets.
struct SrcRows {
  const float *X, *T;
  int64_t rows;
  int in_dim, out_dim;
  __device__ void fill(int64_t tile, int c, int g, bf16x8 &F, float tgt[4], bool &ok) const {
    const int64_t row = 16 * tile + c;
    ok = row < rows;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      const float v = (ok && k < in_dim) ? X[row * in_dim + k] : (k == in_dim ? 1.f : 0.f);
      F[j] = (__bf16)v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) tgt[r] = (ok && r < out_dim) ? T[row * out_dim + r] : 0.f;
  }
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

struct SrcFhn {
  const float *traj;        // [n_traj][S][2 J J]
  const float *ys;          // [n_traj][dy]
  const int32_t *nearest;   // [J J]
  const int32_t *obs_idx;   // [dy]
  int J, S, dy, n_traj, step;
  Key key;
  float tsv, tsw;           // sd / sqrt(h) of v and w
  __device__ void fill(int64_t tile, int c, int g, bf16x8 &F, float tgt[4], bool &ok) const {
    const int nn = J * J, tiles = nn / 16;
    const uint4 w = philox((uint32_t)tile, 0xFFFFFFFCu, (uint32_t)step, P_TRAIN << 24, key);
    const int r = (int)(((uint64_t)w.x * (uint64_t)n_traj) >> 32);
    const int k = (int)(w.y % (uint32_t)S);
    const int node = 16 * (int)(((uint64_t)w.z * (uint64_t)tiles) >> 32) + c;
    ok = true;
    const float *x = traj + ((size_t)r * S + k) * (size_t)(2 * nn);
    const int i = node / J, jj = node - i * J;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int s = 8 * g + j;
      float v;
      if (s < 18) {
        const int q = s < 9 ? s : s - 9;
        const int ni = clampi(i + q / 3 - 1, 0, J - 1), nj = clampi(jj + q % 3 - 1, 0, J - 1);
        v = x[(s < 9 ? 0 : nn) + ni * J + nj];
      } else if (s == 18) {
        const int o = nearest[node];
        v = ys[(size_t)r * dy + o] - x[obs_idx[o]];
      } else if (s == 20 || s == 21) {
        const int ob = obs_idx[nearest[node]];
        v = 0.5f * (float)(s == 20 ? ob / J - i : ob % J - jj);
      } else {
        v = s == 19 ? (float)(S - k) / (float)S : (s == LEARNED_FEATURES ? 1.f : 0.f);
      }
      F[j] = (__bf16)v;
    }
    float z[4];
    normals4(philox((uint32_t)r, 0xFFFFFFFDu, (uint32_t)k, (P_TRAIN << 24) | (uint32_t)(node >> 1), key), z);
    const int e = node & 1;
    tgt[0] = tsv * z[2 * e];
    tgt[1] = tsw * z[2 * e + 1];
    tgt[2] = tgt[3] = 0.f;
  }
};

// 4 rows (4 g .. 4 g + 3) of column `col` of a bf16 tile with row stride `ld`
__device__ __forceinline__ bf16x4 col4(const __bf16 *t, int ld, int g, int col) {
  bf16x4 o;
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] = t[(4 * g + r) * ld + col];
  return o;
}
__device__ __forceinline__ void put4(__bf16 *t, int ld, int row, int col0, const f32x4 &v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) t[row * ld + col0 + r] = (__bf16)v[r];
}

template <class Src>
__global__ void __launch_bounds__(TR_THREADS)
k_mlp_grad(const float *__restrict__ p, int in_dim, int out_dim, Src src, int64_t ntiles,
           float inv_rows, float *__restrict__ partial, int np) {
  __shared__ __bf16 tiles[TR_WAVES * WAVE_LDS];
  __shared__ float w3s[4 * HID];  // bfloat16-rounded W3 (FP32), rows >= out_dim zero
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, c = lane & 15, g = lane >> 4;
  const float *W1 = p, *b1 = W1 + HID * in_dim, *W2 = b1 + HID, *b2 = W2 + HID * HID;
  const float *W3 = b2 + HID;
  (void)b1; (void)b2;
  MlpRegs w;
  mlp_load(p, in_dim, out_dim, w);
  // A operand of the layer-2 backward: row u (input unit) of W2^T, K slots in
  // the hidden order of the forward B operand
  bf16x8 a2t[4][2];
#pragma unroll
  for (int ub = 0; ub < 4; ++ub)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) a2t[ub][kb][j] = (__bf16)W2[hid_slot(kb, g, j) * HID + 16 * ub + c];
  for (int i = tid; i < 4 * HID; i += TR_THREADS)
    w3s[i] = (i / HID) < out_dim ? bf16r(W3[i]) : 0.f;
  __bf16 *h1t = tiles + wid * WAVE_LDS, *da2t = h1t + 16 * LROW, *da1t = da2t + 16 * LROW;
  __bf16 *h2t = da1t + 16 * LROW, *xt = h2t + 16 * LROW, *dt = xt + 16 * XROW;
  // padded outputs of the error tile stay zero
  for (int i = lane; i < 16 * DROW; i += 64) dt[i] = (__bf16)0.f;
  __syncthreads();

  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 gW2[4][4], gW1[4][2], gW3[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = z4;
    gW1[a][0] = gW1[a][1] = z4;
    gW3[a] = z4;
  }
  float gb2[4][4] = {}, gb3[4] = {}, lsum = 0.f;

  const int64_t waves = (int64_t)gridDim.x * TR_WAVES;
  const int64_t iters = (ntiles + waves - 1) / waves;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t tile = (it * gridDim.x + blockIdx.x) * TR_WAVES + wid;
    bf16x8 F;
    float tg[4];
    bool ok = false;
    if (tile < ntiles) {
      src.fill(tile, c, g, F, tg, ok);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) F[j] = (__bf16)0.f;
      tg[0] = tg[1] = tg[2] = tg[3] = 0.f;
    }
    // forward, keeping the pre-activations
    f32x4 a1[4], a2[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) a1[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a1[b], F, z4, 0, 0, 0);
    const bf16x8 h1[2] = {relu_pack(a1[0], a1[1]), relu_pack(a1[2], a1[3])};
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      a2[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a2[ob][0], h1[0], w.b2[ob], 0, 0, 0);
      a2[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a2[ob][1], h1[1], a2[ob], 0, 0, 0);
    }
    const bf16x8 h2[2] = {relu_pack(a2[0], a2[1]), relu_pack(a2[2], a2[3])};
    f32x4 o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a3[0], h2[0], w.b3, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a3[1], h2[1], o, 0, 0, 0);
    // output error d = 2 (u - target) / B on the lanes of group 0 (row c)
    float d[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float e = (ok && r < out_dim && g == 0) ? o[r] - tg[r] : 0.f;
      lsum = fmaf(e, e, lsum);
      d[r] = 2.f * e * inv_rows;
      gb3[r] += d[r];
    }
    float dr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dr[r] = __shfl(d[r], c, 64);  // row c's error to every group
    // layer 3 backward on the VALU, masked by the layer-2 ReLU
    f32x4 da2[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * b + 4 * g + r;
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) s = fmaf(w3s[q * HID + u], dr[q], s);
        da2[b][r] = a2[b][r] > 0.f ? s : 0.f;
        gb2[b][r] += da2[b][r];
      }
    const bf16x8 da2p[2] = {[&] {
                              bf16x8 t;
#pragma unroll
                              for (int r = 0; r < 4; ++r) {
                                t[r] = (__bf16)da2[0][r];
                                t[4 + r] = (__bf16)da2[1][r];
                              }
                              return t;
                            }(),
                            [&] {
                              bf16x8 t;
#pragma unroll
                              for (int r = 0; r < 4; ++r) {
                                t[r] = (__bf16)da2[2][r];
                                t[4 + r] = (__bf16)da2[3][r];
                              }
                              return t;
                            }()};
    // layer 2 backward on MFMA: dh1^T = W2^T . da2^T, masked by the layer-1 ReLU
    f32x4 da1[4];
#pragma unroll
    for (int ub = 0; ub < 4; ++ub) {
      f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2t[ub][0], da2p[0], z4, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2t[ub][1], da2p[1], t, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) da1[ub][r] = a1[ub][r] > 0.f ? t[r] : 0.f;
    }
    // stage the row-major tiles [row c][unit]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f32x4 hv, h2v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        hv[r] = relu(a1[b][r]);
        h2v[r] = relu(a2[b][r]);
      }
      put4(h1t, LROW, c, 16 * b + 4 * g, hv);
      put4(h2t, LROW, c, 16 * b + 4 * g, h2v);
      put4(da2t, LROW, c, 16 * b + 4 * g, da2[b]);
      put4(da1t, LROW, c, 16 * b + 4 * g, da1[b]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) xt[c * XROW + 8 * g + j] = F[j];
    if (g == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dt[c * DROW + r] = (__bf16)d[r];
    }
    __syncthreads();
    // weight gradients: C[unit out][unit in] += A[unit out][rows] B[rows][unit in]
    bf16x4 A_d2[4], A_d1[4], B_h1[4], B_h2[4], B_x[2];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      A_d2[b] = col4(da2t, LROW, g, 16 * b + c);
      A_d1[b] = col4(da1t, LROW, g, 16 * b + c);
      B_h1[b] = col4(h1t, LROW, g, 16 * b + c);
      B_h2[b] = col4(h2t, LROW, g, 16 * b + c);
    }
    B_x[0] = col4(xt, XROW, g, c);
    B_x[1] = col4(xt, XROW, g, 16 + c);
    const bf16x4 A_do = col4(dt, DROW, g, c);
    __syncthreads();
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
      for (int ub = 0; ub < 4; ++ub)
        gW2[jb][ub] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A_d2[jb], B_h1[ub], gW2[jb][ub], 0, 0, 0);
      gW1[jb][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A_d1[jb], B_x[0], gW1[jb][0], 0, 0, 0);
      gW1[jb][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A_d1[jb], B_x[1], gW1[jb][1], 0, 0, 0);
      gW3[jb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A_do, B_h2[jb], gW3[jb], 0, 0, 0);
    }
  }

  // this wave's partial gradient, in the parameter order
  float *out = partial + ((size_t)blockIdx.x * TR_WAVES + wid) * (size_t)(np + 1);
  float *oW1 = out, *ob1 = oW1 + HID * in_dim, *oW2 = ob1 + HID, *ob2 = oW2 + HID * HID;
  float *oW3 = ob2 + HID, *ob3 = oW3 + out_dim * HID;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * jb + 4 * g + r;
#pragma unroll
      for (int ub = 0; ub < 4; ++ub) oW2[j * HID + 16 * ub + c] = gW2[jb][ub][r];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const int k = 16 * kb + c;
        if (k < in_dim) oW1[j * in_dim + k] = gW1[jb][kb][r];
        else if (k == in_dim) ob1[j] = gW1[jb][kb][r];
      }
      const int cc = 4 * g + r;  // output row of the layer-3 product
      if (cc < out_dim) oW3[cc * HID + 16 * jb + c] = gW3[jb][r];
    }
  // bias sums over the 16 rows (lanes c) of each group
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = gb2[b][r];
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
      if (c == 0) ob2[16 * b + 4 * g + r] = v;
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float v = gb3[r];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0 && r < out_dim) ob3[r] = v;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
  if (lane == 0) out[np] = lsum * inv_rows;
}

// grad[i] = sum over waves w of partial[w * stride + i], and the loss from
// slot np when `loss` is given; then, if `adam`, one Adam step of the FP32
// parameters with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t.
// A workgroup takes 64 consecutive parameters; its 16 wave slices sum every
// 16th wave's partial (coalesced rows) and the slices are combined in LDS in
// a fixed order, so the result does not depend on scheduling.
constexpr int RED_SLICES = 16;

__global__ void __launch_bounds__(64 * RED_SLICES)
k_grad_reduce_adam(const float *__restrict__ partial, int nwaves, int stride, int np,
                   float *__restrict__ grad, float *__restrict__ loss, float *__restrict__ p,
                   float *__restrict__ mo, float *__restrict__ ve, float lr, float beta1,
                   float beta2, float omb1, float omb2, float eps, float c1, float c2, int adam) {
  __shared__ float sh[RED_SLICES][64];
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const bool valid = i < np || (i == np && loss);
  float s = 0.f;
  if (valid)
    for (int w = sl; w < nwaves; w += RED_SLICES) s += partial[(size_t)w * stride + i];
  sh[sl][lane] = s;
  __syncthreads();
  if (sl != 0 || !valid) return;
  s = 0.f;
#pragma unroll
  for (int k = 0; k < RED_SLICES; ++k) s += sh[k][lane];
  if (i == np) {
    *loss = s;
    return;
  }
  if (grad) grad[i] = s;
  if (adam) {
    const float m1 = beta1 * mo[i] + omb1 * s;
    const float v1 = beta2 * ve[i] + omb2 * s * s;
    mo[i] = m1;
    ve[i] = v1;
    p[i] -= lr * (m1 / c1) / (sqrtf(v1 / c2) + eps);
  }
}

// ---- FH-N training paths ------------------------------------------------------
constexpr int SIM_THREADS = 320;

__device__ __forceinline__ int hidx(int J, int node) {
  const int i = node / J, j = node - i * J;
  return (i + 1) * (J + 2) + (j + 1);
}
__device__ __forceinline__ void put_v(float *pv, int J, int node, float v) {
  const int i = node / J, j = node - i * J, W = J + 2, hi = (i + 1) * W + (j + 1);
  pv[hi] = v;
  if (i == 0) pv[hi - W] = v;
  if (i == J - 1) pv[hi + W] = v;
  if (j == 0) pv[hi - 1] = v;
  if (j == J - 1) pv[hi + 1] = v;
}

// mode 0 (runs): block q draws x_0 ~ tau_0 and runs run_len intervals,
//   writing x at each interval end to out[q * run_len + j];
// mode 1 (trajectories): block r starts from in[r], writes the state before
//   each step k to out[r][k] and the observation of its end to ys[r].
template <int PPT>
__global__ void __launch_bounds__(SIM_THREADS)
k_train_sim(ModelDev md, Key key, int mode, int count, int run_len, const float *__restrict__ in,
            float *__restrict__ out, float *__restrict__ ys) {
  extern __shared__ float pl[];  // [2][(J+2)^2] v planes
  const int J = md.J, nn = J * J, np = nn / 2, H2 = (J + 2) * (J + 2), W = J + 2;
  const int tid = threadIdx.x;
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const uint32_t c1 = mode == 0 ? 0xFFFFFFFEu : 0xFFFFFFFDu;
    float sv[PPT][2], sw[PPT][2], cv[PPT][2], cw[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int pr = tid + k * SIM_THREADS;
      if (pr < np) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int node = 2 * pr + e;
          if (mode == 0) {
            float z[4];
            normals4(philox((uint32_t)q, c1, 0xFFFFFFFFu, (P_TRAIN << 24) | (uint32_t)(node >> 2), key), z);
            sv[k][e] = md.prior_mean[node] + md.prior_sd[node] * z[node & 3];
            normals4(philox((uint32_t)q, c1, 0xFFFFFFFFu, (P_TRAIN << 24) | (uint32_t)((nn + node) >> 2), key), z);
            sw[k][e] = md.prior_mean[nn + node] + md.prior_sd[nn + node] * z[(nn + node) & 3];
          } else {
            const float *x = in + (size_t)q * 2 * nn;
            sv[k][e] = x[node];
            sw[k][e] = x[nn + node];
          }
          cv[k][e] = cw[k][e] = 0.f;
          put_v(pl, J, node, sv[k][e]);
        }
      }
    }
    __syncthreads();
    const int nsteps = mode == 0 ? run_len * md.S : md.S;
    int cur = 0;
    for (int n = 0; n < nsteps; ++n) {
      float *dst = nullptr;
      if (mode == 1) dst = out + ((size_t)q * md.S + n) * 2 * nn;  // state before step n
      const float *pc = pl + cur * H2;
      float *pn = pl + (cur ^ 1) * H2;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int pr = tid + k * SIM_THREADS;
        if (pr < np) {
          if (dst) {
            *(float2 *)(dst + 2 * pr) = make_float2(sv[k][0], sv[k][1]);
            *(float2 *)(dst + nn + 2 * pr) = make_float2(sw[k][0], sw[k][1]);
          }
          float z[4];
          normals4(philox((uint32_t)q, c1, (uint32_t)n, (P_TRAIN << 24) | (uint32_t)pr, key), z);
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int hi = hidx(J, 2 * pr + e);
            const float cc = sv[k][e];
            const float lap = (((pc[hi - W] - cc) + (pc[hi + W] - cc)) + (pc[hi - 1] - cc)) + (pc[hi + 1] - cc);
            float nv, nw;
            fhn_node_step<false>(md, cc, sw[k][e], lap, z[2 * e], z[2 * e + 1], 0.f, 0.f, nv, nw,
                                 cv[k][e], cw[k][e]);
            sv[k][e] = nv;
            sw[k][e] = nw;
            put_v(pn, J, 2 * pr + e, nv);
          }
        }
      }
      __syncthreads();
      cur ^= 1;
      if (mode == 0 && (n + 1) % md.S == 0) {
        float *o = out + ((size_t)q * run_len + (n + 1) / md.S - 1) * 2 * nn;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          const int pr = tid + k * SIM_THREADS;
          if (pr < np) {
            *(float2 *)(o + 2 * pr) = make_float2(sv[k][0], sv[k][1]);
            *(float2 *)(o + nn + 2 * pr) = make_float2(sw[k][0], sw[k][1]);
          }
        }
      }
    }
    if (mode == 1) {
      const float *pc = pl + cur * H2;
      for (int o = tid; o < md.dy; o += SIM_THREADS) {
        float z[4];
        normals4(philox((uint32_t)q, c1, 0xFFFFFFFFu, (P_TRAIN << 24) | (uint32_t)(o >> 2), key), z);
        ys[(size_t)q * md.dy + o] = pc[hidx(J, md.obs_idx[o])] + md.obs_sd * z[o & 3];
      }
    }
    __syncthreads();
  }
}

int grad_blocks(int64_t ntiles) {
  // about 4 tiles per wave, at most 256 workgroups
  const int64_t b = (ntiles + 4 * TR_WAVES - 1) / (4 * TR_WAVES);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256));
}

}  // namespace

size_t mlp_grad_work_floats(int64_t ntiles, int np) {
  return (size_t)grad_blocks(ntiles) * TR_WAVES * (size_t)(np + 1);
}

// Partial gradients of the allocation-free gradient entry point: one copy
// per device, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it passes the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) float scratch[MLP_GRAD_SCRATCH_BYTES / sizeof(float)];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t mlp_grad_scratch(float **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[dev] = (float *)p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_mlp_grad_rows(const float *params, int in_dim, int out_dim, const float *X,
                                const float *T, int64_t rows, float *partial, float *grad,
                                float *loss, hipStream_t s) {
  const int np = mlp_nparams(in_dim, out_dim);
  const int64_t ntiles = (rows + 15) / 16;
  const int blocks = grad_blocks(ntiles);
  const SrcRows src{X, T, rows, in_dim, out_dim};
  hipLaunchKernelGGL(k_mlp_grad<SrcRows>, dim3(blocks), dim3(TR_THREADS), 0, s, params, in_dim,
                     out_dim, src, ntiles, 1.f / (float)std::max<int64_t>(rows, 1), partial, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_reduce_adam, dim3((np + 1 + 63) / 64), dim3(64 * RED_SLICES), 0, s,
                     partial, blocks * TR_WAVES, np + 1, np, grad, loss, nullptr, nullptr, nullptr, 0.f,
                     0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 0);
  return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *mo, float *ve, int n, double lr,
                       double beta1, double beta2, double eps, int t, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow(beta1, t));
  const float c2 = (float)(1.0 - std::pow(beta2, t));
  hipLaunchKernelGGL(k_grad_reduce_adam, dim3((n + 63) / 64), dim3(64 * RED_SLICES), 0, s, grad, 1,
                     n, n,
                     nullptr, nullptr, params, mo, ve, (float)lr, (float)beta1, (float)beta2,
                     (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps, c1, c2, 1);
  return hipGetLastError();
}

hipError_t launch_train_fhn_step(const ModelDev &md, Key key, const float *traj, const float *ys,
                                 const int32_t *nearest, int n_traj, int step, int batch_tiles,
                                 float tsv, float tsw, float *params, float *partial, float *mo,
                                 float *ve, double lr, double beta1, double beta2, double eps,
                                 float *loss, float *grad, int adam, hipStream_t s) {
  const int np = mlp_nparams(LEARNED_FEATURES, 2);
  const int blocks = grad_blocks(batch_tiles);
  const SrcFhn src{traj, ys, nearest, md.obs_idx, md.J, md.S, md.dy, n_traj, step, key, tsv, tsw};
  hipLaunchKernelGGL(k_mlp_grad<SrcFhn>, dim3(blocks), dim3(TR_THREADS), 0, s, params,
                     LEARNED_FEATURES, 2, src,
                     (int64_t)batch_tiles, 1.f / (16.f * (float)batch_tiles), partial, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float c1 = (float)(1.0 - std::pow(beta1, step));
  const float c2 = (float)(1.0 - std::pow(beta2, step));
  hipLaunchKernelGGL(k_grad_reduce_adam, dim3((np + 1 + 63) / 64), dim3(64 * RED_SLICES), 0, s,
                     partial, blocks * TR_WAVES, np + 1, np, grad, loss, params, mo, ve, (float)lr,
                     (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2),
                     (float)eps, c1, c2, adam);
  return hipGetLastError();
}

hipError_t launch_train_sim(const ModelDev &md, Key key, int mode, int count, int run_len,
                            const float *in, float *out, float *ys, hipStream_t s) {
  const int np = md.J * md.J / 2, ppt = (np + SIM_THREADS - 1) / SIM_THREADS;
  const size_t lds = sizeof(float) * 2 * (size_t)(md.J + 2) * (md.J + 2);
  const dim3 grid((unsigned)std::min(count, 4096));
#define LAUNCH_SIM(P)                                                                        \
  hipLaunchKernelGGL(k_train_sim<P>, grid, dim3(SIM_THREADS), lds, s, md, key, mode, count, \
                     run_len, in, out, ys)
  if (ppt <= 1)
    LAUNCH_SIM(1);
  else if (ppt <= 2)
    LAUNCH_SIM(2);
  else if (ppt <= 4)
    LAUNCH_SIM(4);
  else if (ppt <= 7)
    LAUNCH_SIM(7);
  else
    return hipErrorInvalidValue;
#undef LAUNCH_SIM
  return hipGetLastError();
}

}  // namespace pfk
