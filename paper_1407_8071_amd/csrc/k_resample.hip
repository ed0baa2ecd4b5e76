// k_resample.hip -- normalisation, cumulative weights, sorted uniforms and the
// ancestor search of multinomial resampling (Algorithm 1, steps 2(a)-(b)),
// tiled so that one filter of any N spreads over ceil(N / 4096) workgroups.
//
// Each filter's N log-weights are cut into tiles of 4096 (256 threads x 16
// consecutive elements).  The CDF is held in two levels: a tile-local
// inclusive scan Cl (FP64) and per-tile offsets coff, folded in tile order so
// that coff[q+1] = coff[q] + Cl[last of tile q] holds exactly (the same FP64
// addition): C_i = coff[tile(i)] + Cl[i] is non-decreasing across every tile
// boundary and equals the next tile's offset at the last element of a tile.  The exponential spacings use the
// same two-level layout (Sl, soff).  Uniforms come from exponential spacings:
// E_j = -ln u_j (j = 0..N), S_k = sum_{j<=k} E_j, U_k = S_k / S_N, which are
// the order statistics of N uniforms, so the ancestors come out ascending.
#include <algorithm>

#include "pf_internal.h"

namespace pfk {
namespace {

__device__ __forceinline__ float sane_lw(float v) { return (v == v) ? v : -INFINITY; }

// Tile maximum of the log-weights, as the tile's order-preserving key (0 when
// every weight of the tile is zero).  The fused path's propagation raises the
// same keys as it writes the log-weights, and this launch is then skipped.
__global__ void __launch_bounds__(TILE_THREADS)
k_tile_maxkey(int N, int T, const float *__restrict__ lw, uint32_t *__restrict__ key) {
  __shared__ float sh[TILE_THREADS / 64];
  const int m = blockIdx.y, q = blockIdx.x;
  float v = -INFINITY;
  for (int e = 0; e < TILE_PER_THREAD; ++e) {
    const int i = q * TILE + e * TILE_THREADS + threadIdx.x;
    if (i < N) v = fmaxf(v, sane_lw(lw[(size_t)m * N + i]));
  }
  v = block_max(v, sh);
  if (threadIdx.x == 0) key[(size_t)m * T + q] = v > -INFINITY ? ord_key(v) : 0u;
}

// mx of a filter from its tile maxima (exact, order-free).
__device__ __forceinline__ double filter_max(const uint32_t *__restrict__ key, int m, int T,
                                             float *sh) {
  float v = -INFINITY;
  for (int q = threadIdx.x; q < T; q += blockDim.x) v = fmaxf(v, key_float(key[(size_t)m * T + q]));
  return (double)block_max(v, sh);
}

// Tile-local inclusive scans, one launch: the CDF of w_i = exp(lw_i - mx) in
// FP64 (w = 1 for every particle when no weight is positive), and the sums
// of the exponential variates E_j (the last tile also adds E_N to its
// total).  1024 threads per tile, thread t owning the 4 consecutive
// elements [4t, 4t+4) (one Philox call): with a tile per workgroup a
// single-filter launch has few workgroups, and 16 waves per workgroup hide
// the latency of the FP64 exponentials and logarithms.  The exponentials
// come first since they need no other launch's result.  With X (the fused
// path) it also sums the weighted particles w_i x_i of the tile for the
// weighted estimator (D <= 3 components, component-major [M][D][N]).
constexpr int CDF_THREADS = 1024, CDF_PER_THREAD = TILE / CDF_THREADS;
static_assert(CDF_PER_THREAD % 4 == 0, "whole Philox calls per thread");
__global__ void __launch_bounds__(CDF_THREADS)
k_cdf_uniform_tiles(Key key, int N, int T, int t_arg, const int *tp, const float *__restrict__ lw,
                    const uint32_t *__restrict__ mxkey, double *__restrict__ tile,
                    double *__restrict__ Cl, double *__restrict__ Sl, const float *__restrict__ X,
                    int D, double *__restrict__ wpart) {
  const int t = tp ? *tp : t_arg;
  __shared__ float shf[CDF_THREADS / 64];
  __shared__ double shd[3 * (CDF_THREADS / 64)];
  const int m = blockIdx.y, q = blockIdx.x;
  const int base = q * TILE + threadIdx.x * CDF_PER_THREAD;
  // exponential variates first: they need no other launch's result
  double s[CDF_PER_THREAD];
  double srun = 0.0;
#pragma unroll
  for (int g = 0; g < CDF_PER_THREAD / 4; ++g) {
    const int j0 = base + 4 * g;
    uint4 r = make_uint4(0, 0, 0, 0);
    if (j0 < N) r = philox<2, 3>((uint32_t)(j0 >> 2), (uint32_t)m, (uint32_t)t, P_RESAMPLE << 24, key);
    const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if (j0 + l < N) srun += -log(u01d(rw[l]));
      s[4 * g + l] = srun;
    }
  }
  const double mx = filter_max(mxkey, m, T, shf);
  const bool deg = !(mx > -INFINITY);
  double w[CDF_PER_THREAD];
  double run = 0.0, sq = 0.0, wx[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < CDF_PER_THREAD; ++e) {
    const int i = base + e;
    double we = 0.0;
    if (i < N) we = deg ? 1.0 : exp((double)sane_lw(lw[(size_t)m * N + i]) - mx);
    run += we;
    sq += we * we;
    w[e] = run;
    if (X && i < N)
      for (int c = 0; c < D; ++c) wx[c] += we * (double)X[((size_t)m * D + c) * N + i];
  }
  double tot, stot;
  const double off = block_exscan(run, shd, &tot);
  const double soffv = block_exscan(srun, shd, &stot);
  const int last = min(N - 1, q * TILE + TILE - 1);
#pragma unroll
  for (int e = 0; e < CDF_PER_THREAD; ++e) {
    const int i = base + e;
    if (i < N) {
      const double c = off + w[e];
      Cl[(size_t)m * N + i] = c;
      const double cs = soffv + s[e];
      Sl[(size_t)m * N + i] = cs;
      if (i == last) {
        tile[((size_t)m * T + q) * TREC + 1] = c;
        double tail = 0.0;
        if (q == T - 1) {
          const uint4 r = philox<10, 10>((uint32_t)(N >> 2), (uint32_t)m, (uint32_t)t, P_RESAMPLE << 24, key);
          const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
          tail = -log(u01d(rw[N & 3]));
        }
        tile[((size_t)m * T + q) * TREC + 3] = cs + tail;
      }
    }
  }
  const double s2 = block_sum(sq, shd);
  if (threadIdx.x == 0) tile[((size_t)m * T + q) * TREC + 2] = s2;
  if (X) {
    block_sum_multi_t0<3>(wx, shd);
    if (threadIdx.x == 0)
      for (int c = 0; c < D; ++c) wpart[((size_t)m * T + q) * D + c] = wx[c];
  }
}

// Per filter (one workgroup): tile offsets of the CDF and of the exponential
// sums, the normaliser, ESS and the log G_t^N update of (eqGtN):
// log G += mx + log(W / N) - (d_y/2) log(2 pi s^2).  The offsets are folded
// in tile order by one thread, coff[q+1] = coff[q] + Cl[last of tile q] with
// the very additions the searches repeat, so the two-level CDF is
// non-decreasing across every tile boundary (a tree-ordered scan could leave
// an offset one rounding above or below that sum, and a search could then
// pick a zero-weight particle at a boundary).  The workgroup stages chunks of
// the tile records in LDS for it.
constexpr int FOLD_CHUNK = 1024;
__global__ void __launch_bounds__(256)
k_filter_reduce(int N, int T, double lognorm, const double *__restrict__ tile,
                uint32_t *__restrict__ mxkey, double *__restrict__ coff,
                double *__restrict__ soff, double *__restrict__ fstat) {
  __shared__ double shd[8];
  __shared__ float shf[8];
  __shared__ double cbuf[FOLD_CHUNK], ebuf[FOLD_CHUNK];
  const int m = blockIdx.x;
  const double *rec = tile + (size_t)m * T * TREC;
  double *co = coff + (size_t)m * (T + 1), *so = soff + (size_t)m * (T + 1);
  float lm = -INFINITY;
  double s2 = 0.0;
  for (int q = threadIdx.x; q < T; q += blockDim.x) {
    lm = fmaxf(lm, key_float(mxkey[(size_t)m * T + q]));
    s2 += rec[(size_t)q * TREC + 2];
  }
  const double mx = (double)block_max(lm, shf);
  s2 = block_sum(s2, shd);
  // every thread has read the keys: cleared for the next interval
  for (int q = threadIdx.x; q < T; q += blockDim.x) mxkey[(size_t)m * T + q] = 0u;
  double cc = 0.0, sc = 0.0;  // thread 0's running offsets
  for (int base = 0; base < T; base += FOLD_CHUNK) {
    const int n = min(FOLD_CHUNK, T - base);
    __syncthreads();  // the previous chunk has been folded
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      cbuf[j] = rec[(size_t)(base + j) * TREC + 1];
      ebuf[j] = rec[(size_t)(base + j) * TREC + 3];
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < n; ++j) {
        co[base + j] = cc;
        so[base + j] = sc;
        cc += cbuf[j];
        sc += ebuf[j];
      }
  }
  if (threadIdx.x == 0) {
    co[T] = cc;
    so[T] = sc;
    double *f = fstat + (size_t)m * FREC;
    const bool deg = !(mx > -INFINITY);
    f[0] = mx;
    f[1] = cc;
    f[2] = s2;
    f[3] = deg ? 1.0 : 0.0;
    f[4] = sc;
    f[5] = deg ? -INFINITY : f[5] + mx + log(cc / (double)N) + lognorm;
    f[6] = cc * cc / s2;
  }
}

struct Cdf2 {
  const double *Cl, *coff;
  int N;
  __device__ __forceinline__ double at(int i) const { return coff[i / TILE] + Cl[i]; }
};

// Smallest i in [lo, N-1] with C(i) > v, given C(lo - 1) <= v: exponential
// search from lo, then bisection.  The answer is clamped to N - 1.  (Cdf:
// the two-level CDF with its tile offsets in global memory or in LDS.)
template <class Cdf>
__device__ __forceinline__ int gallop(const Cdf &c, int lo, double v) {
  const int hi_max = c.N - 1;
  if (lo >= hi_max) return hi_max;
  if (c.at(lo) > v) return lo;
  int step = 1, known_le = lo, hi = lo;
  while (true) {
    hi = known_le + step;
    if (hi >= hi_max) {
      hi = hi_max;
      break;
    }
    if (c.at(hi) > v) break;
    known_le = hi;
    step <<= 1;
  }
  int a = known_le + 1, b = hi;  // answer in [a, b]
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (c.at(mid) > v)
      b = mid;
    else
      a = mid + 1;
  }
  return a;
}

// Ancestor a_k = min{ i : C_i > U_k C_{N-1} } for the 16 consecutive k of
// each thread: bisection for the first, exponential search onward.
__global__ void __launch_bounds__(TILE_THREADS)
k_ancestors(int N, int T, const double *__restrict__ Cl, const double *__restrict__ coff,
            const double *__restrict__ Sl, const double *__restrict__ soff,
            const double *__restrict__ fstat, int32_t *__restrict__ A) {
  const int m = blockIdx.y, q = blockIdx.x;
  const int base = q * TILE + threadIdx.x * TILE_PER_THREAD;
  if (base >= N) return;
  const double W = fstat[(size_t)m * FREC + 1];
  const double SN = fstat[(size_t)m * FREC + 4];
  const double so = soff[(size_t)m * (T + 1) + q];
  const Cdf2 c{Cl + (size_t)m * N, coff + (size_t)m * (T + 1), N};
  int i = 0;
  // first target: full bisection
  {
    const double v = ((so + Sl[(size_t)m * N + base]) / SN) * W;
    int a = 0, b = N - 1;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (c.at(mid) > v)
        b = mid;
      else
        a = mid + 1;
    }
    i = a;
    A[(size_t)m * N + base] = i;
  }
  for (int e = 1; e < TILE_PER_THREAD; ++e) {
    const int k = base + e;
    if (k >= N) break;
    const double v = ((so + Sl[(size_t)m * N + k]) / SN) * W;
    i = gallop(c, i, v);
    A[(size_t)m * N + k] = i;
  }
}

// The same ancestors with the tile offsets of the CDF in LDS and 4
// consecutive k per thread (a 256-thread workgroup covers 1024 k, so each
// thread's chain of dependent searches is short): the first search of a
// thread finds the tile by bisection over the offsets in LDS (the offset
// after tile q is C at its last element), then bisects within that tile;
// the others gallop onward.  The result is the same smallest i with
// C_i > U_k C_{N-1} (clamped to N - 1): the offset after tile q is exactly
// coff[q] + Cl[last of q], the value the search inside tile q compares, so
// the tile chosen always holds the answer.
constexpr int ANC_LDS_TILES = 4096;  // tile offsets held in LDS: N <= 4096 * TILE

struct Cdf2L {
  const double *Cl;
  const double *co;  // LDS
  int N;
  __device__ __forceinline__ double at(int i) const { return co[i / TILE] + Cl[i]; }
};

__global__ void __launch_bounds__(TILE_THREADS)
k_ancestors_lds(int N, int T, const double *__restrict__ Cl, const double *__restrict__ coff,
                const double *__restrict__ Sl, const double *__restrict__ soff,
                const double *__restrict__ fstat, int32_t *__restrict__ A) {
  __shared__ double co[ANC_LDS_TILES + 1];
  const int m = blockIdx.y;
  const double *cof = coff + (size_t)m * (T + 1);
  for (int j = threadIdx.x; j <= T; j += TILE_THREADS) co[j] = cof[j];
  __syncthreads();
  const int base = blockIdx.x * ANC_SPAN + threadIdx.x * ANC_PER_THREAD;
  if (base >= N) return;
  const double W = fstat[(size_t)m * FREC + 1];
  const double SN = fstat[(size_t)m * FREC + 4];
  const double so = soff[(size_t)m * (T + 1) + base / TILE];  // the 4 k share a tile
  const double *cl = Cl + (size_t)m * N;
  const Cdf2L c{cl, co, N};
  int i;
  {
    const double v = ((so + Sl[(size_t)m * N + base]) / SN) * W;
    int a = 0, b = T - 1;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (co[mid + 1] > v)
        b = mid;
      else
        a = mid + 1;
    }
    const double off = co[a];
    int lo = a * TILE, hi = min(N - 1, (a + 1) * TILE - 1);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (off + cl[mid] > v)
        hi = mid;
      else
        lo = mid + 1;
    }
    i = lo;
    A[(size_t)m * N + base] = i;
  }
#pragma unroll
  for (int e = 1; e < ANC_PER_THREAD; ++e) {
    const int k = base + e;
    if (k >= N) break;
    const double v = ((so + Sl[(size_t)m * N + k]) / SN) * W;
    i = gallop(c, i, v);
    A[(size_t)m * N + k] = i;
  }
}

// The fused path's ancestor search for filters of at most FOLD_MAX_TILES
// tiles, with the per-filter fold inside it: every workgroup folds the
// filter's tile totals into the CDF and spacing offsets in LDS (one thread,
// in tile order -- the additions of k_filter_reduce, so every workgroup holds
// the same offsets and the two-level CDF is non-decreasing across tile
// boundaries), the filter's first workgroup writes its record (mx, W, sum w^2,
// S_N, log G_t^N, ESS) and clears its tile maximum keys, and each workgroup
// sums the post-resampling particles x^(a_k) of its 1024 k for the
// estimator (span partial sums, folded with the cross-filter means).  Search
// as in k_ancestors_lds.
template <int D>
__global__ void __launch_bounds__(TILE_THREADS)
k_ancestors_fold(int N, int T, int G, double lognorm, const double *__restrict__ tile,
                 uint32_t *__restrict__ mxkey, const double *__restrict__ Cl,
                 const double *__restrict__ Sl, double *__restrict__ fstat,
                 int32_t *__restrict__ A, const float *__restrict__ X,
                 double *__restrict__ mpart) {
  // (tile totals and offsets in separate arrays, so that the fold's loads
  // run ahead of its stores)
  __shared__ double ct[FOLD_MAX_TILES], st[FOLD_MAX_TILES];
  __shared__ double co[FOLD_MAX_TILES + 1], so[FOLD_MAX_TILES + 1];
  __shared__ double shd[D * (TILE_THREADS / 64)];
  __shared__ float shf[TILE_THREADS / 64];
  const int m = blockIdx.y;
  // Workgroup b = blockIdx.x + G m runs on XCD b mod 8, and resampling tile
  // q of filter m was formed on XCD (q + T m) mod 8 (workgroup q + T m of
  // the CDF launch).  The span of targets g lies mostly in tile g / 4
  // (ANC_SPAN = TILE / 4), so where G is a multiple of 32 each workgroup
  // takes a span of the tiles formed on its own XCD (a bijection of the
  // spans), and its searches read that XCD's L2.
  int g = blockIdx.x;
  if (G % 32 == 0 && 4 * ANC_SPAN == TILE) {
    const int r = g & 7, a = g >> 3;
    const int x = (int)(((long)r + (long)(G - T) * m) & 7);
    g = 32 * (a >> 2) + 4 * x + (a & 3);
  }
  const double *rec = tile + (size_t)m * T * TREC;
  for (int j = threadIdx.x; j < T; j += TILE_THREADS) {
    ct[j] = rec[(size_t)j * TREC + 1];
    st[j] = rec[(size_t)j * TREC + 3];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double cc = 0.0, sc = 0.0;
#pragma unroll 8
    for (int j = 0; j < T; ++j) {
      co[j] = cc;
      so[j] = sc;
      cc += ct[j];
      sc += st[j];
    }
    co[T] = cc;
    so[T] = sc;
  }
  __syncthreads();
  const double W = co[T], SN = so[T];
  if (g == 0) {
    float lm = -INFINITY;
    double s2 = 0.0;
    for (int q = threadIdx.x; q < T; q += TILE_THREADS) {
      lm = fmaxf(lm, key_float(mxkey[(size_t)m * T + q]));
      s2 += rec[(size_t)q * TREC + 2];
    }
    const double mx = (double)block_max(lm, shf);
    s2 = block_sum(s2, shd);
    // every thread has read the keys: cleared for the next interval
    for (int q = threadIdx.x; q < T; q += TILE_THREADS) mxkey[(size_t)m * T + q] = 0u;
    if (threadIdx.x == 0) {
      double *f = fstat + (size_t)m * FREC;
      const bool deg = !(mx > -INFINITY);
      f[0] = mx;
      f[1] = W;
      f[2] = s2;
      f[3] = deg ? 1.0 : 0.0;
      f[4] = SN;
      f[5] = deg ? -INFINITY : f[5] + mx + log(W / (double)N) + lognorm;
      f[6] = W * W / s2;
    }
  }
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  const int base = g * ANC_SPAN + threadIdx.x * ANC_PER_THREAD;
  if (base < N) {
    const double sot = so[base / TILE];  // the 4 k share a tile
    const double *cl = Cl + (size_t)m * N;
    const Cdf2L c{cl, co, N};
    auto take = [&](int k, int i) {
      A[(size_t)m * N + k] = i;
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d] += (double)X[((size_t)m * D + d) * N + i];
    };
    int i;
    {
      const double v = ((sot + Sl[(size_t)m * N + base]) / SN) * W;
      int a = 0, b = T - 1;
      while (a < b) {
        const int mid = (a + b) >> 1;
        if (co[mid + 1] > v)
          b = mid;
        else
          a = mid + 1;
      }
      const double off = co[a];
      int lo = a * TILE, hi = min(N - 1, (a + 1) * TILE - 1);
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (off + cl[mid] > v)
          hi = mid;
        else
          lo = mid + 1;
      }
      i = lo;
      take(base, i);
    }
#pragma unroll
    for (int e = 1; e < ANC_PER_THREAD; ++e) {
      const int k = base + e;
      if (k >= N) break;
      const double v = ((sot + Sl[(size_t)m * N + k]) / SN) * W;
      i = gallop(c, i, v);
      take(k, i);
    }
  }
  block_sum_multi_t0<D>(acc, shd);
  if (threadIdx.x == 0)
#pragma unroll
    for (int d = 0; d < D; ++d) mpart[((size_t)m * G + g) * D + d] = acc[d];
}

// Per-filter means from the tile partial sums (one workgroup per filter,
// fixed summation order), then the equal-weight ensemble average of
// Definition 3 in the next kernel.
__global__ void __launch_bounds__(256)
k_filter_means(int N, int T, int dx, const double *__restrict__ mpart,
               const double *__restrict__ wpart, const double *__restrict__ fstat,
               double *__restrict__ fmean, double *__restrict__ fmeanw) {
  __shared__ double sh[8];
  const int m = blockIdx.x;
  const double W = fstat[(size_t)m * FREC + 1];
  for (int c = 0; c < dx; ++c) {
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < T; q += blockDim.x) {
      a += mpart[((size_t)m * T + q) * dx + c];
      b += wpart[((size_t)m * T + q) * dx + c];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
      fmean[(size_t)m * dx + c] = a / (double)N;
      fmeanw[(size_t)m * dx + c] = b / W;
    }
  }
}

__global__ void __launch_bounds__(256)
k_ensemble_mean(int M, int dx, const double *__restrict__ fmean, const double *__restrict__ fmeanw,
                double *__restrict__ emean) {
  __shared__ double sh[4];
  if (dx <= 64) {
    // few components: the workgroup reduces over filters for each component
    for (int c = 0; c < dx; ++c) {
      double a = 0.0, b = 0.0;
      for (int m = threadIdx.x; m < M; m += blockDim.x) {
        a += fmean[(size_t)m * dx + c];
        b += fmeanw[(size_t)m * dx + c];
      }
      a = block_sum(a, sh);
      b = block_sum(b, sh);
      if (threadIdx.x == 0) {
        emean[c] = a / (double)M;
        emean[dx + c] = b / (double)M;
      }
    }
  } else {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= dx) return;
    double a = 0.0, b = 0.0;
    for (int m = 0; m < M; ++m) {
      a += fmean[(size_t)m * dx + c];
      b += fmeanw[(size_t)m * dx + c];
    }
    emean[c] = a / (double)M;
    emean[dx + c] = b / (double)M;
  }
}

// One workgroup per ensemble: equal-weight average of its filters' means.
// (256 threads, or 1024 where an ensemble has more filters; for dx <= 3 every
// thread takes all 2 dx sums over its filters in one pass, and one block
// reduction folds them.)
__global__ void __launch_bounds__(1024)
k_ensemble_means_batched(const FusedEns *__restrict__ ens, int *t_inc) {
  __shared__ double sh[16];
  __shared__ double shm[6 * 16];
  // every earlier kernel of the interval has read the counter
  if (t_inc && blockIdx.x == 0 && threadIdx.x == 0) *t_inc += 1;
  const FusedEns &E = ens[blockIdx.x];
  // grid models (both FH-N forms): folded by their own state-wide estimator
  if (E.md.kind >= 2) return;
  const int dx = E.md.dx;
  if (E.mpart) {
    // a tiled ensemble: its filters' means from the estimator's partial sums
    // (post-resampling ones per ancestor span, weighted ones per tile); a
    // group of waves per filter, each wave summing every component over a
    // strided share of the partials, the group's sums added in LDS
    __shared__ double part[16][6];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int per = max(1, nw / E.M);  // waves per filter
    for (int m0 = 0; m0 < E.M; m0 += nw / per) {
      const int m = m0 + wid / per, sub = wid % per;
      const bool on = wid / per < nw / per && m < E.M;
      double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
      if (on) {
        for (int j = sub * 64 + lane; j < E.G; j += per * 64)
          for (int c = 0; c < dx; ++c) a[c] += gptr(E.mpart)[((size_t)m * E.G + j) * dx + c];
        for (int j = sub * 64 + lane; j < E.T; j += per * 64)
          for (int c = 0; c < dx; ++c) b[c] += gptr(E.wpart)[((size_t)m * E.T + j) * dx + c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a[c] = wave_sum(a[c]);
        b[c] = wave_sum(b[c]);
      }
      if (lane == 0)
        for (int c = 0; c < 3; ++c) {
          part[wid][c] = a[c];
          part[wid][3 + c] = b[c];
        }
      __syncthreads();
      if (on && sub == 0 && lane < 2 * dx) {
        const int c = lane % dx, r = lane < dx ? c : 3 + c;
        double v = 0.0;
        for (int k = 0; k < per; ++k) v += part[wid + k][r];
        if (lane < dx)
          gptr(E.fmean)[(size_t)m * dx + c] = v / (double)E.N;
        else
          gptr(E.fmeanw)[(size_t)m * dx + c] = v / gptr(E.fstat)[(size_t)m * FREC + 1];
      }
      __syncthreads();  // (part is reused; the filter means are read below)
    }
  }
  if (dx <= 3) {
    double v[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = 0.0;
    for (int m = threadIdx.x; m < E.M; m += blockDim.x) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < dx) {
          v[c] += gptr(E.fmean)[(size_t)m * dx + c];
          v[3 + c] += gptr(E.fmeanw)[(size_t)m * dx + c];
        }
    }
    block_sum_multi_t0<6>(v, shm);
    if (threadIdx.x == 0)
      for (int c = 0; c < dx; ++c) {
        gptr(E.emean)[c] = v[c] / (double)E.M;
        gptr(E.emean)[dx + c] = v[3 + c] / (double)E.M;
      }
    return;
  }
  for (int c = 0; c < dx; ++c) {
    double a = 0.0, b = 0.0;
    for (int m = threadIdx.x; m < E.M; m += blockDim.x) {
      a += gptr(E.fmean)[(size_t)m * dx + c];
      b += gptr(E.fmeanw)[(size_t)m * dx + c];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
      gptr(E.emean)[c] = a / (double)E.M;
      gptr(E.emean)[dx + c] = b / (double)E.M;
    }
  }
}

}  // namespace

hipError_t launch_ensemble_means(const FusedEns *d_ens, int n_ens, int max_m, bool tiled,
                                 int *t_inc, hipStream_t s) {
  // 1024 threads for many filters, or where the partial sums of more than
  // four tiled filters are folded (a wave per filter, in one round)
  if (n_ens > 0)
    k_ensemble_means_batched<<<n_ens, (max_m > 256 || tiled) ? 1024 : 256, 0, s>>>(d_ens, t_inc);
  return hipGetLastError();
}

namespace {
__global__ void k_set_i32(int *p, int v) { *p = v; }

__global__ void __launch_bounds__(256) k_fill_f32(float *p, float v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    p[i] = v;
}
}  // namespace

// a one-thread kernel instead of a memset, so that it is safe in graphs
hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  k_fill_f32<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_set_i32(int *p, int v, hipStream_t s) {
  k_set_i32<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_resample(const EnsDev &e, int t, hipStream_t s, const int *tp) {
  const dim3 g((unsigned)e.T, (unsigned)e.M);
  k_tile_maxkey<<<g, TILE_THREADS, 0, s>>>(e.N, e.T, e.lw, e.mxkey);
  k_cdf_uniform_tiles<<<g, CDF_THREADS, 0, s>>>(e.key, e.N, e.T, t, tp, e.lw, e.mxkey, e.tile, e.Cl,
                                                 e.Sl, nullptr, 0, nullptr);
  k_filter_reduce<<<e.M, 256, 0, s>>>(e.N, e.T, e.lognorm, e.tile, e.mxkey, e.coff, e.soff,
                                      e.fstat);
  if (e.T <= ANC_LDS_TILES) {
    const dim3 ga((unsigned)((e.N + ANC_SPAN - 1) / ANC_SPAN), (unsigned)e.M);
    k_ancestors_lds<<<ga, TILE_THREADS, 0, s>>>(e.N, e.T, e.Cl, e.coff, e.Sl, e.soff, e.fstat, e.A);
  } else {
    k_ancestors<<<g, TILE_THREADS, 0, s>>>(e.N, e.T, e.Cl, e.coff, e.Sl, e.soff, e.fstat, e.A);
  }
  return hipGetLastError();
}

hipError_t launch_resample_fused(const EnsDev &e, IvArg iv, const float *X, bool key_ready,
                                 hipStream_t s) {
  if (e.T > FOLD_MAX_TILES || e.md.dx > 3) return hipErrorInvalidValue;
  const dim3 g((unsigned)e.T, (unsigned)e.M);
  if (!key_ready) k_tile_maxkey<<<g, TILE_THREADS, 0, s>>>(e.N, e.T, e.lw, e.mxkey);
  k_cdf_uniform_tiles<<<g, CDF_THREADS, 0, s>>>(e.key, e.N, e.T, iv.t, iv.tp, e.lw, e.mxkey, e.tile,
                                                 e.Cl, e.Sl, X, e.md.dx, e.wpart);
  const int G = (e.N + ANC_SPAN - 1) / ANC_SPAN;
  const dim3 ga((unsigned)G, (unsigned)e.M);
  if (e.md.dx == 3)
    k_ancestors_fold<3><<<ga, TILE_THREADS, 0, s>>>(e.N, e.T, G, e.lognorm, e.tile, e.mxkey, e.Cl,
                                                     e.Sl, e.fstat, e.A, X, e.mpart);
  else
    k_ancestors_fold<1><<<ga, TILE_THREADS, 0, s>>>(e.N, e.T, G, e.lognorm, e.tile, e.mxkey, e.Cl,
                                                     e.Sl, e.fstat, e.A, X, e.mpart);
  return hipGetLastError();
}

hipError_t launch_combine_means(const EnsDev &e, bool ensemble_mean, hipStream_t s) {
  const int dx = e.md.dx;
  k_filter_means<<<e.M, 256, 0, s>>>(e.N, e.T, dx, e.mpart, e.wpart, e.fstat, e.fmean, e.fmeanw);
  if (!ensemble_mean) return hipGetLastError();
  const unsigned g = dx <= 64 ? 1u : (unsigned)((dx + 255) / 256);
  k_ensemble_mean<<<g, 256, 0, s>>>(e.M, dx, e.fmean, e.fmeanw, e.emean);
  return hipGetLastError();
}

}  // namespace pfk
