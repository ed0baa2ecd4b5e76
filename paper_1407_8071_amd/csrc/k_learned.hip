// k_learned.hip -- the learned proposal on gfx950: a drift correction
// u_theta(features) added to every Euler-Maruyama increment, with the
// particle's weight multiplied by the exact ratio of the model and proposal
// increment densities (the importance-function form of the filter that the
// paper's closing remarks of Sec. 6 extend its results to).
//
// The network and its MFMA mapping are in mlp_device.h.
#include <algorithm>
#include <cmath>

#include "mlp_device.h"

namespace pfk {
namespace {

// ---------------------------------------------------------------------------
// u_theta over the rows of X [rows][in_dim] -> out [rows][out_dim].
constexpr int FWD_THREADS = 256;

__global__ void __launch_bounds__(FWD_THREADS)
k_mlp_forward(const float *__restrict__ p, int in_dim, int out_dim, const float *__restrict__ X,
              int64_t rows, float *__restrict__ out) {
  MlpRegs w;
  mlp_load(p, in_dim, out_dim, w);
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
  const int64_t ntiles = (rows + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (FWD_THREADS / 64) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (FWD_THREADS / 64);
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    const int64_t row = 16 * t + c;
    const bool ok = row < rows;
    bf16x8 F;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      const float v = (ok && k < in_dim) ? X[row * in_dim + k] : (k == in_dim ? 1.f : 0.f);
      F[j] = (__bf16)v;
    }
    const f32x4 o = mlp_tile(w, F);
    if (g == 0 && ok) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < out_dim) out[row * out_dim + r] = o[r];
    }
  }
}

// ---------------------------------------------------------------------------
// One observation interval of FH-N particles under the learned proposal.
//
// A workgroup owns one particle at a time, with both planes in LDS inside a
// one-node halo that replicates the edge (which is both the edge replication
// of the 3x3 feature patch and the no-flux truncation of the Laplacian: an
// outside neighbour equals the node, so its term is exactly +0).  Per Euler
// step: (A) every wave runs MLP tiles of 16 consecutive nodes (features from
// the current planes) and stores (u_v, u_w) of each node in LDS; (B) every
// thread advances its node pairs (Philox call of pair p at step n, the same
// counters as the bootstrap kernels) with the drift correction, accumulates
// the log increment-density ratio, and writes the other plane buffer.  Two
// barriers per step.  The first read goes through the ancestors (fused
// gather); the last step ends with the log-weight: observation term plus the
// accumulated ratio.
//
// LDS (floats): planes [2 buffers][v, w][(J+2)^2], u [2][J*J], y of the
// nearest observation [J*J], halo index of that observation [J*J] (int),
// 32 of reduction scratch.
constexpr int LS_THREADS = 320;  // 5 waves

struct LearnedConst {
  float c1v, c2v, c1w, c2w;  // sqrt(h)/sd and h/(2 sd^2) per variable class
};

__device__ __forceinline__ void put_node(float *pl, int H2, int J, int node, float v, float w) {
  const int i = node / J, j = node - i * J, W = J + 2;
  const int hi = (i + 1) * W + (j + 1);
  float *pv = pl, *pw = pl + H2;
  pv[hi] = v;
  pw[hi] = w;
  const bool top = i == 0, bot = i == J - 1, lef = j == 0, rig = j == J - 1;
  if (top) { pv[hi - W] = v; pw[hi - W] = w; }
  if (bot) { pv[hi + W] = v; pw[hi + W] = w; }
  if (lef) { pv[hi - 1] = v; pw[hi - 1] = w; }
  if (rig) { pv[hi + 1] = v; pw[hi + 1] = w; }
  if (top && lef) { pv[hi - W - 1] = v; pw[hi - W - 1] = w; }
  if (top && rig) { pv[hi - W + 1] = v; pw[hi - W + 1] = w; }
  if (bot && lef) { pv[hi + W - 1] = v; pw[hi + W - 1] = w; }
  if (bot && rig) { pv[hi + W + 1] = v; pw[hi + W + 1] = w; }
}

__device__ __forceinline__ int halo_index(int J, int node) {
  const int i = node / J, j = node - i * J;
  return (i + 1) * (J + 2) + (j + 1);
}

template <int PPT>
__global__ void __launch_bounds__(LS_THREADS)
k_grid_steps_learned(ModelDev md, Key key, int M, int N, IvArg iv, int yoff,
                     const float *__restrict__ Xin, const int32_t *__restrict__ anc,
                     float *__restrict__ Xout, float *__restrict__ lw,
                     const float *__restrict__ params, const int32_t *__restrict__ nearest,
                     LearnedConst lc) {
  extern __shared__ float lds[];
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t) + yoff;
  const int J = md.J, nn = J * J, np = nn / 2, W = J + 2, H2 = W * W;
  float *planes = lds;                    // [2][2][H2]
  float *U = lds + 4 * H2;                // [2][nn]
  float *YN = U + 2 * nn;                 // [nn]
  int *ON = (int *)(YN + nn);             // [nn]
  float *red = (float *)(ON + nn);        // [32]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, c = lane & 15, g = lane >> 4;
  const int nwaves = LS_THREADS / 64, ntiles = (nn + 15) / 16;

  MlpRegs w;
  mlp_load(params, LEARNED_FEATURES, 2, w);
  // feature slots 8 g + j of this lane: patch offsets into the current buffer
  // (v plane, then w plane), or a constant (tau, 1, 0) for the others; the
  // residual and the observation offsets (slots 18, 20, 21) are filled in
  // per node below
  int fo[8];
  bool frel[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * g + j;
    if (k < 18) {
      const int q = k < 9 ? k : k - 9;
      fo[j] = (k < 9 ? 0 : H2) + (q / 3 - 1) * W + (q % 3 - 1);
      frel[j] = true;
    } else {
      fo[j] = 0;
      frel[j] = k == 18;  // the residual: replaced below
    }
  }
  // per node: y of the nearest observation, and its halo index (bits 0-15)
  // with its row and column offsets + 128 (bits 16-23, 24-31)
  for (int n = tid; n < nn; n += LS_THREADS) {
    const int o = nearest[n], ob = md.obs_idx[o];
    YN[n] = y[o];
    const int di = ob / J - n / J, dj = ob % J - n % J;
    ON[n] = halo_index(J, ob) | ((di + 128) << 16) | ((dj + 128) << 24);
  }

  for (int p = blockIdx.x; p < M * N; p += gridDim.x) {
    const int m = p / N, i = p - m * N;
    const int src = anc ? min(max(anc[(size_t)m * N + i], 0), N - 1) : i;
    const float *in = Xin + ((size_t)m * N + src) * (2 * nn);
    float sv[PPT][2], sw[PPT][2], cv[PPT][2], cw[PPT][2];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pr = tid + q * LS_THREADS;
      if (pr < np) {
        const float2 a = *(const float2 *)(in + 2 * pr);
        const float2 b = *(const float2 *)(in + nn + 2 * pr);
        sv[q][0] = a.x; sv[q][1] = a.y; sw[q][0] = b.x; sw[q][1] = b.y;
        cv[q][0] = cv[q][1] = cw[q][0] = cw[q][1] = 0.f;
        put_node(planes, H2, J, 2 * pr, a.x, b.x);
        put_node(planes, H2, J, 2 * pr + 1, a.y, b.y);
      }
    }
    __syncthreads();
    float dl = 0.f;
    int cur = 0;
    const int n0 = (t - 1) * md.S;
    for (int st = 0; st < md.S; ++st) {
      const float tau = (float)(md.S - st) / (float)md.S;
      const float *pc = planes + cur * 2 * H2;
      // (A) drift corrections of every node
      for (int tt = wid; tt < ntiles; tt += nwaves) {
        const int node = min(16 * tt + c, nn - 1);
        const int ctr = halo_index(J, node);
        bf16x8 F;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = 8 * g + j;
          const float cst = k == 19 ? tau : (k == LEARNED_FEATURES ? 1.f : 0.f);
          F[j] = (__bf16)(frel[j] ? pc[ctr + fo[j]] : cst);
        }
        if (g == 2) {
          const unsigned on = (unsigned)ON[node];
          F[2] = (__bf16)(YN[node] - pc[on & 0xFFFFu]);
          F[4] = (__bf16)(0.5f * (float)((int)((on >> 16) & 0xFFu) - 128));
          F[5] = (__bf16)(0.5f * (float)((int)(on >> 24) - 128));
        }
        const f32x4 o = mlp_tile(w, F);
        if (g == 0 && 16 * tt + c < nn) {
          U[16 * tt + c] = o[0];
          U[nn + 16 * tt + c] = o[1];
        }
      }
      __syncthreads();
      // (B) Euler-Maruyama with the corrected drift
      float *pn = planes + (cur ^ 1) * 2 * H2;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int pr = tid + q * LS_THREADS;
        if (pr < np) {
          float z[4];
          normals4(philox((uint32_t)i, (uint32_t)m, (uint32_t)(n0 + st),
                          (P_PROP << 24) | (uint32_t)pr, key), z);
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int node = 2 * pr + e;
            const int hi = halo_index(J, node);
            const float cc = sv[q][e];
            const float lap = (((pc[hi - W] - cc) + (pc[hi + W] - cc)) + (pc[hi - 1] - cc)) +
                              (pc[hi + 1] - cc);
            const float uv = U[node], uw = U[nn + node];
            const float zv = z[2 * e], zw = z[2 * e + 1];
            float nv, nw;
            fhn_node_step<true>(md, cc, sw[q][e], lap, zv, zw, uv, uw, nv, nw, cv[q][e], cw[q][e]);
            sv[q][e] = nv;
            sw[q][e] = nw;
            dl += (-(lc.c1v * uv * zv) - lc.c2v * uv * uv) + (-(lc.c1w * uw * zw) - lc.c2w * uw * uw);
          }
          put_node(pn, H2, J, 2 * pr, sv[q][0], sw[q][0]);
          put_node(pn, H2, J, 2 * pr + 1, sv[q][1], sw[q][1]);
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    // state out, then the log-weight: observation term + density ratio
    float *out = Xout + ((size_t)m * N + i) * (2 * nn);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pr = tid + q * LS_THREADS;
      if (pr < np) {
        *(float2 *)(out + 2 * pr) = make_float2(sv[q][0], sv[q][1]);
        *(float2 *)(out + nn + 2 * pr) = make_float2(sw[q][0], sw[q][1]);
      }
    }
    if (lw) {
      const float *pc = planes + cur * 2 * H2;
      float acc = 0.f;
      for (int k = tid; k < md.dy; k += LS_THREADS) {
        const float r = y[k] - pc[halo_index(J, md.obs_idx[k])];
        acc = fmaf(r, r, acc);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, 64);
        dl += __shfl_xor(dl, o, 64);
      }
      if (lane == 0) {
        red[wid] = acc;
        red[16 + wid] = dl;
      }
      __syncthreads();
      if (tid == 0) {
        float a = 0.f, d = 0.f;
        for (int k = 0; k < nwaves; ++k) {
          a += red[k];
          d += red[16 + k];
        }
        const float l = -a * md.inv2var + d;
        lw[(size_t)m * N + i] = (l == l) ? l : -INFINITY;
      }
    }
    __syncthreads();
  }
}

}  // namespace

size_t learned_lds_bytes(int J) {
  const size_t H2 = (size_t)(J + 2) * (J + 2), nn = (size_t)J * J;
  return sizeof(float) * (4 * H2 + 4 * nn + 32);
}

hipError_t set_learned_lds_limit() {
  const int bytes = (int)learned_lds_bytes(48);
  const void *fs[4] = {(const void *)k_grid_steps_learned<1>, (const void *)k_grid_steps_learned<2>,
                       (const void *)k_grid_steps_learned<3>, (const void *)k_grid_steps_learned<4>};
  for (const void *f : fs) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int learned_resident_blocks(int J) {
  const int np = J * J / 2, ppt = (np + LS_THREADS - 1) / LS_THREADS;
  const size_t lds = learned_lds_bytes(J);
  int per_cu = 0, dev = 0, cus = 256;
  const void *f = ppt <= 1 ? (const void *)k_grid_steps_learned<1>
                  : ppt <= 2 ? (const void *)k_grid_steps_learned<2>
                  : ppt <= 3 ? (const void *)k_grid_steps_learned<3>
                             : (const void *)k_grid_steps_learned<4>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, LS_THREADS, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

hipError_t launch_mlp_forward(const float *params, int in_dim, int out_dim, const float *X,
                              int64_t rows, float *out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t tiles = (rows + 15) / 16;
  const int64_t waves = (int64_t)FWD_THREADS / 64;
  const int blocks = (int)std::min<int64_t>((tiles + waves - 1) / waves, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(FWD_THREADS), 0, s, params, in_dim, out_dim,
                     X, rows, out);
  return hipGetLastError();
}

hipError_t launch_grid_steps_learned(const EnsDev &e, IvArg iv, int yoff, const float *Xin,
                                     const int32_t *anc, float *Xout, float *lw,
                                     const float *params, const int32_t *nearest, double sd0,
                                     double sd1, int blocks, hipStream_t s) {
  const ModelDev &md = e.md;
  if (!iv.y || md.kind != 2) return hipErrorInvalidValue;
  const int np = md.J * md.J / 2;
  const int ppt = (np + LS_THREADS - 1) / LS_THREADS;
  const double h = md.h;
  const LearnedConst lc{(float)(std::sqrt(h) / sd0), (float)(h / (2.0 * sd0 * sd0)),
                        (float)(std::sqrt(h) / sd1), (float)(h / (2.0 * sd1 * sd1))};
  const size_t lds = learned_lds_bytes(md.J);
  const int MN = e.M * e.N;
  const dim3 grid((unsigned)std::min(MN, blocks));
#define LAUNCH_LS(P)                                                                        \
  hipLaunchKernelGGL(k_grid_steps_learned<P>, grid, dim3(LS_THREADS), lds, s, md, e.key, e.M, \
                     e.N, iv, yoff, Xin, anc, Xout, lw, params, nearest, lc)
  if (ppt <= 1)
    LAUNCH_LS(1);
  else if (ppt <= 2)
    LAUNCH_LS(2);
  else if (ppt <= 3)
    LAUNCH_LS(3);
  else if (ppt <= 4)
    LAUNCH_LS(4);
  else
    return hipErrorInvalidValue;
#undef LAUNCH_LS
  return hipGetLastError();
}

}  // namespace pfk
