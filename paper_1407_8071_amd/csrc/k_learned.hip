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
  Mlp32Regs w;
  mlp32_load(p, in_dim, out_dim, w);
  const int l = threadIdx.x & 63, c = l & 31, h = l >> 5;
  const int64_t ntiles = (rows + 31) / 32;
  const int64_t wave = (int64_t)blockIdx.x * (FWD_THREADS / 64) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (FWD_THREADS / 64);
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    const int64_t row = 32 * t + c;
    const bool ok = row < rows;
    bf16x8 F[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * kb + 8 * h + j;
        const float v = (ok && k < in_dim) ? X[row * in_dim + k] : (k == in_dim ? 1.f : 0.f);
        F[kb][j] = (__bf16)v;
      }
    const f32x16 o = mlp32_tile(w, F);
    if (h == 0 && ok) {
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
// step: (A) every wave runs MLP tiles of 32 consecutive nodes (features from
// the current planes) and stores (u_v, u_w) of each node in LDS; (B) every
// thread advances its node pairs (Philox call of pair p at step n, the same
// counters as the bootstrap kernels) with the drift correction, accumulates
// the log increment-density ratio, and writes the interior of the other
// plane buffer; (C) the edge nodes are copied into that buffer's halo.  Three
// barriers per step.  The first read goes through the ancestors (fused
// gather); the last step ends with the log-weight: observation term plus the
// accumulated ratio.
//
// LDS (floats): planes [2 buffers][v, w][(J+2)^2], the compensation terms of
// the Euler sums [v, w][J*J], u [2][J*J], y of the nearest observation [J*J],
// that observation's halo index and offsets [J*J] (int), 32 of reduction
// scratch.
constexpr int LS_THREADS = 256;  // 4 waves: two workgroups per CU

struct LearnedConst {
  float c1v, c2v, c1w, c2w;  // sqrt(h)/sd and h/(2 sd^2) per variable class
};

// row of node n = i J + j for n < 4096, J <= 64: (n + 1/2) / J lies at least
// 1/(2J) inside (i, i + 1), far above the rounding of the float product
__device__ __forceinline__ int node_row(int n, float invJ) {
  return (int)(((float)n + 0.5f) * invJ);
}

// Replicate the edge nodes of both planes into the one-node halo (corners
// take the corner node); the interior must be complete and visible.
__device__ __forceinline__ void fill_halo(float *pl, int H2, int J) {
  const int W = J + 2, nh = 2 * W + 2 * J;
  for (int k = threadIdx.x; k < nh; k += LS_THREADS) {
    int r, c;
    if (k < 2 * W) {
      r = k < W ? 0 : W - 1;
      c = k < W ? k : k - W;
    } else {
      r = (k < 2 * W + J ? k - 2 * W : k - 2 * W - J) + 1;
      c = k < 2 * W + J ? 0 : W - 1;
    }
    const int src = min(max(r, 1), J) * W + min(max(c, 1), J), dst = r * W + c;
    pl[dst] = pl[src];
    pl[H2 + dst] = pl[H2 + src];
  }
}

__device__ __forceinline__ int halo_index(int J, int node) {
  const int i = node / J, j = node - i * J;
  return (i + 1) * (J + 2) + (j + 1);
}

__global__ void __launch_bounds__(LS_THREADS, 2)
k_grid_steps_learned(ModelDev md, Key key, int M, int N, IvArg iv, int yoff,
                     const float *__restrict__ Xin, const int32_t *__restrict__ anc,
                     float *__restrict__ Xout, float *__restrict__ lw,
                     const float *__restrict__ params, const int32_t *__restrict__ nearest,
                     LearnedConst lc) {
  extern __shared__ float lds[];
  const int t = iv_t(iv);
  const float *y = iv_y(iv, t) + yoff;
  const int J = md.J, nn = J * J, np = nn / 2, W = J + 2, H2 = W * W;
  const float invJ = 1.f / (float)J;
  float *planes = lds;                    // [2][2][H2]
  float *CMP = lds + 4 * H2;              // [2][nn]
  float *U = CMP + 2 * nn;                // [2][nn]
  float *YN = U + 2 * nn;                 // [nn]
  int *ON = (int *)(YN + nn);             // [nn]
  float *red = (float *)(ON + nn);        // [32]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, c = lane & 15, g = lane >> 4;
  const int nwaves = LS_THREADS / 64, ntiles = (nn + 31) / 32;
  const int c32 = lane & 31, h = lane >> 5;
  (void)c; (void)g;

  Mlp32Regs w;
  mlp32_load(params, LEARNED_FEATURES, 2, w);
  // inputs of lane half h: slots 8 h .. 8 h + 7 (patch values: offsets from
  // the node's halo index, v plane then w plane) and, on half 0, slots
  // 16 .. 23 (the last two w values, residual, tau, observation offsets,
  // the constant 1, 0); half 1 holds zeros in slots 24 .. 31
  int fo[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * h + j;
    const int q = k < 9 ? k : k - 9;
    fo[j] = (k < 9 ? 0 : H2) + (q / 3 - 1) * W + (q % 3 - 1);
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
    for (int pr = tid; pr < np; pr += LS_THREADS) {
      const float2 a = *(const float2 *)(in + 2 * pr);
      const float2 b = *(const float2 *)(in + nn + 2 * pr);
      const int ni = node_row(2 * pr, invJ), nj = 2 * pr - ni * J;
      const int hi = (ni + 1) * W + (nj + 1);
      planes[hi] = a.x;
      planes[hi + 1] = a.y;
      planes[H2 + hi] = b.x;
      planes[H2 + hi + 1] = b.y;
      *(float2 *)(CMP + 2 * pr) = make_float2(0.f, 0.f);
      *(float2 *)(CMP + nn + 2 * pr) = make_float2(0.f, 0.f);
    }
    __syncthreads();
    fill_halo(planes, H2, J);
    __syncthreads();
    float dl = 0.f;
    int cur = 0;
    const int n0 = (t - 1) * md.S;
    for (int st = 0; st < md.S; ++st) {
      const float tau = (float)(md.S - st) / (float)md.S;
      const float *pc = planes + cur * 2 * H2;
      // (A) drift corrections of every node: 32-node MLP tiles per wave; the
      // inputs of the next tile are read while this tile's MFMAs run
      auto inputs = [&](int tt, bf16x8 F[2]) {
        const int node = min(32 * tt + c32, nn - 1);
        const int ni = node_row(node, invJ), nj = node - ni * J;
        const int ctr = (ni + 1) * W + (nj + 1);
#pragma unroll
        for (int j = 0; j < 8; ++j) F[0][j] = (__bf16)pc[ctr + fo[j]];
        const float w7 = pc[ctr + H2 + W], w8 = pc[ctr + H2 + W + 1];
        const unsigned on = (unsigned)ON[node];
        const float res = YN[node] - pc[on & 0xFFFFu];
        const float f1[8] = {w7, w8, res, tau, 0.5f * (float)((int)((on >> 16) & 0xFFu) - 128),
                             0.5f * (float)((int)(on >> 24) - 128), 1.f, 0.f};
#pragma unroll
        for (int j = 0; j < 8; ++j) F[1][j] = (__bf16)(h == 0 ? f1[j] : 0.f);
      };
      bf16x8 Fc[2], Fn[2];
      if (wid < ntiles) inputs(wid, Fc);
      for (int tt = wid; tt < ntiles; tt += nwaves) {
        if (tt + nwaves < ntiles) inputs(tt + nwaves, Fn);
        const f32x16 o = mlp32_tile(w, Fc);
        if (h == 0 && 32 * tt + c32 < nn) {
          U[32 * tt + c32] = o[0];
          U[nn + 32 * tt + c32] = o[1];
        }
        Fc[0] = Fn[0];
        Fc[1] = Fn[1];
      }
      __syncthreads();
      // (B) Euler-Maruyama with the corrected drift; the compensation terms
      // of the sums stay in LDS
      float *pn = planes + (cur ^ 1) * 2 * H2;
      for (int pr = tid; pr < np; pr += LS_THREADS) {
        float z[4];
        normals4(philox((uint32_t)i, (uint32_t)m, (uint32_t)(n0 + st),
                        (P_PROP << 24) | (uint32_t)pr, key), z);
        const int ni = node_row(2 * pr, invJ), nj0 = 2 * pr - ni * J;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int node = 2 * pr + e;
          const int hi = (ni + 1) * W + (nj0 + e + 1);
          const float cc = pc[hi], ww = pc[H2 + hi];
          const float lap = (((pc[hi - W] - cc) + (pc[hi + W] - cc)) + (pc[hi - 1] - cc)) +
                            (pc[hi + 1] - cc);
          const float uv = U[node], uw = U[nn + node];
          const float zv = z[2 * e], zw = z[2 * e + 1];
          float nv, nw, cv = CMP[node], cw = CMP[nn + node];
          fhn_node_step<true>(md, cc, ww, lap, zv, zw, uv, uw, nv, nw, cv, cw);
          CMP[node] = cv;
          CMP[nn + node] = cw;
          dl += (-(lc.c1v * uv * zv) - lc.c2v * uv * uv) + (-(lc.c1w * uw * zw) - lc.c2w * uw * uw);
          pn[hi] = nv;
          pn[H2 + hi] = nw;
        }
      }
      __syncthreads();
      fill_halo(pn, H2, J);
      __syncthreads();
      cur ^= 1;
    }
    // state out, then the log-weight: observation term + density ratio
    const float *pc = planes + cur * 2 * H2;
    float *out = Xout + ((size_t)m * N + i) * (2 * nn);
    for (int pr = tid; pr < np; pr += LS_THREADS) {
      const int ni = node_row(2 * pr, invJ), nj = 2 * pr - ni * J;
      const int hi = (ni + 1) * W + (nj + 1);
      *(float2 *)(out + 2 * pr) = make_float2(pc[hi], pc[hi + 1]);
      *(float2 *)(out + nn + 2 * pr) = make_float2(pc[H2 + hi], pc[H2 + hi + 1]);
    }
    if (lw) {
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
  return sizeof(float) * (4 * H2 + 6 * nn + 32);
}

hipError_t set_learned_lds_limit() {
  return hipFuncSetAttribute((const void *)k_grid_steps_learned,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)learned_lds_bytes(48));
}

int learned_resident_blocks(int J) {
  int per_cu = 0, dev = 0, cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_grid_steps_learned,
                                                   LS_THREADS, learned_lds_bytes(J)) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

hipError_t launch_mlp_forward(const float *params, int in_dim, int out_dim, const float *X,
                              int64_t rows, float *out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t tiles = (rows + 31) / 32;
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
  if (!iv.y || md.kind != 2 || md.J > 48) return hipErrorInvalidValue;
  const double h = md.h;
  const LearnedConst lc{(float)(std::sqrt(h) / sd0), (float)(h / (2.0 * sd0 * sd0)),
                        (float)(std::sqrt(h) / sd1), (float)(h / (2.0 * sd1 * sd1))};
  const int MN = e.M * e.N;
  hipLaunchKernelGGL(k_grid_steps_learned, dim3((unsigned)std::min(MN, blocks)),
                     dim3(LS_THREADS), learned_lds_bytes(md.J), s, md, e.key, e.M, e.N, iv, yoff,
                     Xin, anc, Xout, lw, params, nearest, lc);
  return hipGetLastError();
}

}  // namespace pfk
