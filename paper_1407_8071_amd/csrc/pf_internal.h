// pf_internal.h -- device-buffer views of one ensemble and the host-side
// launchers of every kernel.  Internal to libpf; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf.h"
#include "pf_device.h"

namespace pfk {

// Elements per resampling tile: 256 threads x 16 consecutive elements.
constexpr int TILE_THREADS = 256;
constexpr int TILE_PER_THREAD = 16;
constexpr int TILE = TILE_THREADS * TILE_PER_THREAD;

// Per-tile record (doubles): 0 max lw, 1 sum w (= last local CDF value),
// 2 sum w^2, 3 sum of the tile's exponential variates (incl. E_N on the last).
constexpr int TREC = 4;
// Ancestor searches of the tiled resampler: 4 consecutive k per thread of a
// 256-thread workgroup, so 1024 k per workgroup ("span").
constexpr int ANC_PER_THREAD = 4, ANC_SPAN = TILE_THREADS * ANC_PER_THREAD;
// The fused path folds a filter's tile offsets inside every ancestor
// workgroup up to this many tiles (N <= 4 Mi); larger filters take the
// separate per-filter fold.
constexpr int FOLD_MAX_TILES = 1024;
// Per-filter record (doubles): 0 mx, 1 W, 2 sum w^2, 3 degenerate flag,
// 4 S_N, 5 log G_t^N (running), 6 ESS of the last interval, 7 kept flag
// (FREC_KEPT).
constexpr int FREC = 8;

struct EnsDev {
  ModelDev md;
  Key key;
  uint32_t seed_lo, seed_hi;
  int32_t M, N, T;  // filters, particles, tiles per filter
  double lognorm;   // -(dy/2) log(2 pi obs_var)
  float *X[2];      // particle buffers
  float *lw;        // [M][N]
  int32_t *A;       // [M][N]
  double *Cl;       // [M][N] tile-local inclusive CDF
  double *Sl;       // [M][N] tile-local inclusive sums of exponentials
  double *tile;     // [M][T][TREC]
  uint32_t *mxkey;  // [M][T] order-preserving key of each tile's maximum log-weight (0: empty)
  double *coff;     // [M][T+1] CDF tile offsets
  double *soff;     // [M][T+1] exponential-sum tile offsets
  double *fstat;    // [M][FREC]
  double *mpart;    // [M][G][dx] partial sums of post-resampling particles (G = spans >= T)
  double *wpart;    // [M][T][dx] partial sums of weighted particles
  double *fmean;    // [M][dx]
  double *fmeanw;   // [M][dx]
  double *emean;    // [2][dx]: ensemble post-resampling and weighted means
};

// Interval index and observations of a fused launch: by value for a direct
// launch, or read from device memory (tp, and y + (t-1) * ystride) so that a
// captured graph replays every interval unchanged.
struct IvArg {
  int t;
  const int *tp;
  const float *y;
  int ystride;
};
__device__ __forceinline__ int iv_t(const IvArg &a) { return a.tp ? *a.tp : a.t; }
__device__ __forceinline__ const float *iv_y(const IvArg &a, int t) {
  return a.y ? a.y + (a.ystride ? (size_t)(t - 1) * a.ystride : 0) : nullptr;
}

// Device-side record of one ensemble for the fused interval kernels.
struct FusedEns {
  ModelDev md;
  Key key;
  int32_t M, N;
  int32_t yoff;  // offset of this ensemble's observations
  double lognorm;
  float *X0, *X1, *lw;
  int32_t *A;
  double *fstat, *fmean, *fmeanw, *emean;
  // grid model: offspring counts [M][N], estimator partials [M][nch][2][dx]
  int32_t *cnt;
  double *gpart;
  int32_t nch;
  // resampling scheme (RS_*), and the ESS-triggered schedule: resample when
  // ESS < ess_thr N (ess_thr > 0); lwc [M][N] holds the carried log-weights
  // of particles that were not resampled (normalised to mean weight 1)
  int32_t scheme;
  double ess_thr;
  float *lwc;
  // auxiliary particle filter: pilot log-likelihoods [M][N] of the particles
  // at the start of the interval (the first stage's weights are lwc + lpil)
  int32_t apf;
  float *lpil;
  // tiled vector ensembles on the fused path (else null): the tile maximum
  // keys that propagation raises, and the estimator's partial sums that the
  // cross-filter means fold -- per ancestor span (post-resampling, G per
  // filter) and per tile (weighted, T per filter)
  uint32_t *mxkey;
  double *mpart, *wpart;
  int32_t T, G;
};
enum { RS_MULTINOMIAL = 0, RS_SYSTEMATIC = 1, RS_STRATIFIED = 2, RS_RESIDUAL = 3 };
// per-filter record slot 7: 1.0 when the last interval kept its particles
// (ESS above the threshold), so that the filter's estimate is the weighted one
constexpr int FREC_KEPT = 7;

// ---- vector models (OU, Lorenz 63): particles [M][dx][N] ------------------
hipError_t launch_vec_init(const EnsDev &e, float *X, hipStream_t s);
hipError_t launch_vec_propagate(const EnsDev &e, int t, const float *Xin, const int32_t *anc,
                                float *Xout, float *lw_or_null, const float *y, hipStream_t s);
hipError_t launch_vec_loglik(const EnsDev &e, const float *X, const float *y, hipStream_t s);
hipError_t launch_vec_gather(const EnsDev &e, const float *Xin, float *Xout, hipStream_t s);
// estimates of the filters: post-resampling particles read from Xpost (through
// `anc` when not null), weighted ones from Xpre; optionally the ensemble mean
hipError_t launch_vec_estimate(const EnsDev &e, const float *Xpost, const float *Xpre,
                               const int32_t *anc, bool ensemble_mean, hipStream_t s);
hipError_t launch_vec_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                               hipStream_t s);

// ---- resampling (any model): lw [M][N] -> A [M][N] ------------------------
hipError_t launch_resample(const EnsDev &e, int t, hipStream_t s, const int *tp = nullptr);
// The fused path's tiled resampling (T <= FOLD_MAX_TILES): the CDF and
// spacings with the weighted estimator's tile sums, then the ancestor search
// with the tile offsets folded in every workgroup, the filter records and
// the post-resampling estimator's span sums; the tile maximum keys come from
// propagation (key_ready) or from a key launch here.
hipError_t launch_resample_fused(const EnsDev &e, IvArg iv, const float *X, bool key_ready,
                                 hipStream_t s);
hipError_t launch_combine_means(const EnsDev &e, bool ensemble_mean, hipStream_t s);

// ---- filter-per-workgroup interval kernel (vector models, N <= WG_MAX_N) ---
constexpr int WG_MAX_N = 8192;
struct WgJob {
  int32_t ens, filter;
};
size_t filter_wg_lds(int N, int BD);
size_t resample_wg_lds(int N, int BD);
hipError_t set_filter_wg_lds_limit();
hipError_t launch_filter_wg(int D, int BD, const WgJob *d_jobs, int n_jobs, int max_n,
                            const FusedEns *d_ens, IvArg iv, int parity, int pending,
                            int resample_only, hipStream_t s);
// resampling of each job's filter from its log-weights; offspring counts to
// d_counts[ensemble] (an array of per-ensemble device pointers)
// stage 0: the interval's resampling (or, for auxiliary filters, the
// normalisation of the second-stage weights, which are carried); stage 1:
// the first-stage resampling of auxiliary filters from their pilot weights
hipError_t launch_resample_wg(int D, int BD, const WgJob *d_jobs, int n_jobs, int max_n,
                              const FusedEns *d_ens, IvArg iv, int32_t *const *d_counts,
                              int xb_parity, bool custom, int stage, hipStream_t s);
// the paper's FH-N network (kind 3): interval t of every particle of fused
// ensemble e (log-weights when iv carries observations), and the truth path
hipError_t launch_fhnp_steps(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s);
hipError_t launch_fhnp_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                                hipStream_t s);
// its auxiliary-filter pilot (S noise-free steps without new stimuli)
hipError_t launch_fhnp_pilot(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s);
// auxiliary filters: the pilot -- the noise-free S-step Euler path of every
// particle and its log-likelihood -- and the first-stage log-weights
hipError_t launch_vec_pilot(int D, const FusedEns *d_ens, int e, int M, int N, IvArg iv,
                            int parity, int pending, hipStream_t s);
hipError_t launch_grid_pilot(const FusedEns *d_ens, int e, int M, int N, int J, IvArg iv,
                             int parity, int pending, hipStream_t s);
// batched propagation + weighting of vector-model tiles {ens, filter, i0, -}
hipError_t launch_vec_prop_batched(int D, const int4 *d_tiles, int n_tiles, int tile_width,
                                  const FusedEns *d_ens, IvArg iv, int parity, int pending,
                                  hipStream_t s);
hipError_t launch_offspring_counts(const EnsDev &e, int32_t *cnt, hipStream_t s);

// ---- grid model (FH-N): particles [M][N][2][J][J] ---------------------------
int grid_resident_blocks(const ModelDev &md);
hipError_t launch_grid_init(const EnsDev &e, float *X, hipStream_t s);
hipError_t launch_grid_stream_step(const EnsDev &e, int n, const float *Xin, const int32_t *anc,
                                   float *Xout, float *lw, const float *y, int blocks,
                                   hipStream_t s);
hipError_t launch_grid_loglik(const EnsDev &e, const float *X, const float *y, hipStream_t s);
hipError_t launch_grid_gather(const EnsDev &e, const float *Xin, float *Xout, hipStream_t s);
int grid_est_chunks(int N);
hipError_t launch_grid_estimate(const EnsDev &e, const float *Xb, const int32_t *cnt,
                                double *part, hipStream_t s);
hipError_t launch_grid_simulate(const EnsDev &e, uint64_t seed, int T, float *xtrue, float *y,
                                hipStream_t s);

// Batched grid model (fused path): every particle of the grid ensembles of
// one grid size J in one launch, from a table of {ensemble, filter, particle}
// entries; the estimator from tables of {ensemble, filter, chunk} and
// {ensemble, filter} jobs and a list of ensembles.
hipError_t launch_grid_steps_batched(int J, const int4 *d_ptab, int n_p, const FusedEns *d_ens,
                                     IvArg iv, int parity, int pending, int blocks, hipStream_t s);
hipError_t launch_grid_estimate_batched(int J, const int4 *d_part_jobs, int n_part,
                                        const int4 *d_fold_jobs, int n_fold, const int *d_gens,
                                        int n_gens, const FusedEns *d_ens, int out, hipStream_t s);
int grid_resident_blocks_j(int J);
// particles per workgroup of the batched stepping kernel (1..8, fixed per J
// and device); its particle table holds each ensemble's entries padded to a
// multiple of this with ensemble -1
int grid_steps_ppb(int J);

// cross-filter averages of many ensembles at once (one workgroup each)
// t_inc (optional): device interval counter advanced once the means are done
// max_m: the largest filter count of the ensembles (sets the workgroup size)
hipError_t launch_ensemble_means(const FusedEns *d_ens, int n_ens, int max_m, bool tiled,
                                 int *t_inc, hipStream_t s);
hipError_t launch_set_i32(int *p, int v, hipStream_t s);
// p[0 .. n) = v (a kernel, not a memset node, so that it may be captured)
hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s);

// ---- learned proposal (MLP in -> 64 -> 64 -> out, FP32 master parameters) ---
constexpr int MLP_HIDDEN = 64;
inline int mlp_nparams(int in_dim, int out_dim) {
  return MLP_HIDDEN * in_dim + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN +
         out_dim * MLP_HIDDEN + out_dim;
}
size_t learned_lds_bytes(int J);
int learned_resident_blocks(int J);
hipError_t set_learned_lds_limit();
hipError_t launch_mlp_forward(const float *params, int in_dim, int out_dim, const float *X,
                              int64_t rows, float *out, hipStream_t s);
// interval of an FH-N ensemble under the learned proposal (needs iv.y);
// nearest[J*J] = index of each node's nearest observation
hipError_t launch_grid_steps_learned(const EnsDev &e, IvArg iv, int yoff, const float *Xin,
                                     const int32_t *anc, float *Xout, float *lw,
                                     const float *params, const int32_t *nearest, double sd0,
                                     double sd1, int blocks, hipStream_t s);

// training of u_theta: partial-gradient buffer size (floats) for ntiles
// tiles of 16 rows, the gradient over explicit rows, Adam, one FH-N training
// step (minibatch from stored trajectories + Adam), the training paths
size_t mlp_grad_work_floats(int64_t ntiles, int np);
// the allocation-free gradient's static partial-gradient buffer: its size,
// and its device address on the current device (looked up on first use)
constexpr size_t MLP_GRAD_SCRATCH_BYTES = PF_MLP_GRAD_STATIC_BYTES;
hipError_t mlp_grad_scratch(float **out);
hipError_t launch_mlp_grad_rows(const float *params, int in_dim, int out_dim, const float *X,
                                const float *T, int64_t rows, float *partial, float *grad,
                                float *loss, hipStream_t s);
hipError_t launch_adam(float *params, const float *grad, float *mo, float *ve, int n, double lr,
                       double beta1, double beta2, double eps, int t, hipStream_t s);
hipError_t launch_train_fhn_step(const ModelDev &md, Key key, const float *traj, const float *ys,
                                 const int32_t *nearest, int n_traj, int step, int batch_tiles,
                                 float tsv, float tsw, float *params, float *partial, float *mo,
                                 float *ve, double lr, double beta1, double beta2, double eps,
                                 float *loss, float *grad, int adam, hipStream_t s);
hipError_t launch_train_sim(const ModelDev &md, Key key, int mode, int count, int run_len,
                            const float *in, float *out, float *ys, hipStream_t s);

// ---- random-number hook ----------------------------------------------------
hipError_t launch_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                                uint32_t *bits, float *z, hipStream_t s);

}  // namespace pfk
