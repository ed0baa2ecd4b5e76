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

__global__ void __launch_bounds__(FWD_THREADS, 2)
k_mlp_forward(const float *__restrict__ p, int in_dim, int out_dim, const float *__restrict__ X,
              int64_t rows, float *__restrict__ out) {
  Mlp32Regs w;
  mlp32_load(p, in_dim, out_dim, w, InputsInOrder{in_dim});
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
    const f32x2 u = mlp32_tile<4>(w, F);
    if (ok && h < out_dim) out[row * out_dim + h] = u[0];
    if (ok && 2 + h < out_dim) out[row * out_dim + 2 + h] = u[1];
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
// the halo indices of the patch corner and of that observation [J*J] (int),
// the observation's offsets [J*J] (bfloat16 pair), 32 of reduction scratch.
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

// Input slots of the FH-N proposal (features in the order of
// fhn_features: v patch 0..8, w patch 9..17, residual, tau, row and column
// offsets).  Lane half h reads patch positions 0..7 of plane h (slots 8 h + j,
// one base address per half); slots 16..23 of half 0 hold v and w at patch
// position 8, the residual, tau, the offsets, the constant 1 and a zero;
// slots 24..31 are zero.
struct FhnSlots {
  __device__ int operator()(int k) const {
    if (k < 8) return k;
    if (k < 16) return 9 + (k - 8);
    constexpr int tail[8] = {8, 17, 18, 19, 20, 21, SLOT_ONE, SLOT_ZERO};
    return k < 24 ? tail[k - 16] : SLOT_ZERO;
  }
};

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
  int *NO = (int *)(YN + nn);             // [nn]
  unsigned *OFF = (unsigned *)(NO + nn);  // [nn]
  float *red = (float *)(OFF + nn);       // [32]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nwaves = LS_THREADS / 64, ntiles = (nn + 31) / 32;
  const int c32 = lane & 31, h = lane >> 5;

  Mlp32Regs w;
  mlp32_load(params, LEARNED_FEATURES, 2, w, FhnSlots{});
  // per node: y of the nearest observation; the halo index of the node's
  // patch corner (bits 0-15) and of that observation (bits 16-31); the
  // observation's row and column offsets / 2 as a bfloat16 pair
  for (int n = tid; n < nn; n += LS_THREADS) {
    const int o = nearest[n], ob = md.obs_idx[o];
    YN[n] = y[o];
    const int ni = n / J, nj = n - ni * J;
    NO[n] = (ni * W + nj) | (halo_index(J, ob) << 16);
    const f32x2 off = {0.5f * (float)(ob / J - ni), 0.5f * (float)(ob % J - nj)};
    OFF[n] = __builtin_bit_cast(unsigned, __builtin_convertvector(off, bf16x2));
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
      // (no = NO of the tile's node, read one tile earlier still, so that no
      // LDS read waits on another)
      auto tile_node = [&](int tt) { return min(32 * tt + c32, nn - 1); };
      // half 1 holds zeros in slots 24..31: an AND with a lane mask (a select
      // would let the compiler move the reads under a branch)
      const unsigned keep = h == 0 ? 0xFFFFFFFFu : 0u;
      const unsigned one_lo = keep & 0x3F80u;  // bfloat16 (1, 0)
      auto inputs = [&](int tt, int no, bf16x8 F[2]) {
        const int node = tile_node(tt), base = no & 0xFFFF;
        const float *r0 = pc + base + h * H2, *r1 = r0 + W, *r2 = r1 + W;
        const float q[8] = {r0[0], r0[1], r0[2], r1[0], r1[1], r1[2], r2[0], r2[1]};
#pragma unroll
        for (int j = 0; j < 8; ++j) F[0][j] = (__bf16)q[j];
        const float v8 = pc[base + 2 * W + 2], w8 = pc[base + H2 + 2 * W + 2];
        const float res = YN[node] - pc[no >> 16];
        const f32x2 a = {v8, w8}, b = {res, tau};
        u32x4 f1;
        f1[0] = keep & __builtin_bit_cast(unsigned, __builtin_convertvector(a, bf16x2));
        f1[1] = keep & __builtin_bit_cast(unsigned, __builtin_convertvector(b, bf16x2));
        f1[2] = keep & OFF[node];
        f1[3] = one_lo;
        F[1] = __builtin_bit_cast(bf16x8, f1);
      };
      // (the read of the next tile is unconditional -- the last one repeats
      // a valid tile -- so that it stays in the MFMA block and its LDS
      // latency hides under the MFMAs)
      // The tiles run at a raised wave priority: where the other workgroup
      // on the CU is in its Euler phase, the SIMD then issues this wave's
      // MFMAs and their packing first and fills the matrix pipe's gaps with
      // the other wave's VALU work, instead of taking both in turn.
      __builtin_amdgcn_s_setprio(2);
      bf16x8 Fc[2], Fn[2];
      int no_n = NO[tile_node(min(wid + nwaves, ntiles - 1))];
      if (wid < ntiles) inputs(wid, NO[tile_node(wid)], Fc);
      for (int tt = wid; tt < ntiles; tt += nwaves) {
        const int no_nn = NO[tile_node(min(tt + 2 * nwaves, ntiles - 1))];
        inputs(min(tt + nwaves, ntiles - 1), no_n, Fn);
        const f32x2 u = mlp32_tile<2>(w, Fc);
        if (32 * tt + c32 < nn) U[h * nn + 32 * tt + c32] = u[0];  // u_v, u_w by lane half
        Fc[0] = Fn[0];
        Fc[1] = Fn[1];
        no_n = no_nn;
      }
      __builtin_amdgcn_s_setprio(0);
      __syncthreads();
      // (B) Euler-Maruyama with the corrected drift; the compensation terms
      // of the sums stay in LDS
      float *pn = planes + (cur ^ 1) * 2 * H2;
      for (int pr = tid; pr < np; pr += LS_THREADS) {
        // every LDS read of the pair first (the stores below go to the other
        // buffer, which the compiler cannot tell apart)
        const int ni = node_row(2 * pr, invJ), nj0 = 2 * pr - ni * J;
        const int hi = (ni + 1) * W + (nj0 + 1);
        const float c0 = pc[hi], c1 = pc[hi + 1], l0 = pc[hi - 1], r1 = pc[hi + 2];
        const float u0 = pc[hi - W], u1 = pc[hi - W + 1], d0 = pc[hi + W], d1 = pc[hi + W + 1];
        const float w0 = pc[H2 + hi], w1 = pc[H2 + hi + 1];
        const float2 uv = *(const float2 *)(U + 2 * pr), uw = *(const float2 *)(U + nn + 2 * pr);
        float2 cv = *(const float2 *)(CMP + 2 * pr), cw = *(const float2 *)(CMP + nn + 2 * pr);
        float z[4];
        normals4(philox<4, 3>((uint32_t)i, (uint32_t)m, (uint32_t)(n0 + st),
                        (P_PROP << 24) | (uint32_t)pr, key), z);
        // node 2 pr: right neighbour c1; node 2 pr + 1: left neighbour c0
        const float lap0 = (((u0 - c0) + (d0 - c0)) + (l0 - c0)) + (c1 - c0);
        const float lap1 = (((u1 - c1) + (d1 - c1)) + (c0 - c1)) + (r1 - c1);
        float nv0, nw0, nv1, nw1;
        fhn_node_step<true>(md, c0, w0, lap0, z[0], z[1], uv.x, uw.x, nv0, nw0, cv.x, cw.x);
        fhn_node_step<true>(md, c1, w1, lap1, z[2], z[3], uv.y, uw.y, nv1, nw1, cv.y, cw.y);
        dl += (-(lc.c1v * uv.x * z[0]) - lc.c2v * uv.x * uv.x) +
              (-(lc.c1w * uw.x * z[1]) - lc.c2w * uw.x * uw.x);
        dl += (-(lc.c1v * uv.y * z[2]) - lc.c2v * uv.y * uv.y) +
              (-(lc.c1w * uw.y * z[3]) - lc.c2w * uw.y * uw.y);
        *(float2 *)(CMP + 2 * pr) = cv;
        *(float2 *)(CMP + nn + 2 * pr) = cw;
        pn[hi] = nv0;
        pn[hi + 1] = nv1;
        pn[H2 + hi] = nw0;
        pn[H2 + hi + 1] = nw1;
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
  return sizeof(float) * (4 * H2 + 7 * nn + 32);
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
