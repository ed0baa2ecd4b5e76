// pf_api.cpp -- the C ABI of include/pf.h: descriptor validation, workspace
// layout, and the per-interval orchestration of the gfx950 kernels.
#include "pf.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pf_internal.h"

namespace {

thread_local std::string g_err;

pf_status fail(pf_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

pf_status dev(hipError_t e, const char *what) {
  if (e == hipSuccess) return PF_OK;
  return fail(PF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define PF_TRY(expr)                  \
  do {                                \
    pf_status _s = (expr);            \
    if (_s != PF_OK) return _s;       \
  } while (0)
#define PF_HIP(expr) PF_TRY(dev((expr), #expr))

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Host-side record of one ensemble.
struct Ens {
  pf_ensemble_desc d;
  int dx, dy, T;
  bool grid;
  bool wg;     // fused path: one filter-per-workgroup kernel does the whole interval
  bool tiled;  // fused path (vector, N > WG_MAX_N): multi-workgroup resampling kernels
  std::vector<int32_t> obs_idx;
  std::vector<float> prior_mean, prior_sd;
  pfk::EnsDev dev;
  pfk::FusedEns fz;  // record of the fused kernels
  int blocks = 1024;       // grid model: resident workgroups of the stepping kernels
  int32_t *cnt = nullptr;  // grid model: offspring counts [M][N]
  double *gpart = nullptr; // grid model: estimator partial sums
  float *lwc = nullptr;    // ESS schedule, auxiliary filter: carried log-weights [M][N]
  bool apf = false;        // auxiliary particle filter
  bool paper = false;      // the paper's FH-N network (kind 3)
  // learned proposal (FH-N): FP32 parameters and each node's nearest observation
  bool learned = false;
  float *params = nullptr;
  int32_t *nearest = nullptr;
  double sd0 = 0.0, sd1 = 0.0;
  int lblocks = 256;
};

// One launch of the filter-per-workgroup kernel: every filter of the
// ensembles of one (state dimension, workgroup size) class.
// kinds of workgroup-per-filter launches
enum { CLASS_FILTER_WG = 0, CLASS_RESAMPLE_VEC = 1, CLASS_RESAMPLE_GRID = 2, CLASS_APF_FIRST = 3 };
struct WgClass {
  int kind;
  int D, BD, max_n;  // D = 0: grid-model resampling class
  bool custom = false;  // resampling classes: another scheme or the ESS schedule
  std::vector<pfk::WgJob> jobs;
  pfk::WgJob *d_jobs = nullptr;
};

// Workgroup size of the filter-per-workgroup kernel for N particles.
// (the per-filter kernels hold one element per thread below 1024 threads)
int wg_block(int N, int bd_min = 256) {
  for (int bd = 64; bd <= 512; bd <<= 1)
    if (bd >= bd_min && N <= bd) return bd;
  return 1024;
}

// Offsets of every array of one ensemble inside the workspace.
struct Layout {
  size_t obs, pmean, psd, X0, X1, lw, A, Cl, Sl, tile, mxkey, coff, soff, fstat, mpart, wpart,
      fmean, fmeanw, emean, cnt, gpart, params, nearest, lwc, lpil, end;
};

constexpr int LEARNED_IN = 22, LEARNED_OUT = 2;  // FH-N node features, (u_v, u_w)
constexpr int LEARNED_MAX_J = 48;

Layout layout_of(size_t base, int M, int N, int dx, int dy, int T, bool grid, bool learned,
                 bool carried, bool auxiliary) {
  Layout L{};
  size_t o = base;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t MN = (size_t)M * N;
  L.obs = take(sizeof(int32_t) * (size_t)dy);
  L.pmean = take(sizeof(float) * (size_t)dx);
  L.psd = take(sizeof(float) * (size_t)dx);
  L.X0 = take(sizeof(float) * MN * dx);
  L.X1 = take(sizeof(float) * MN * dx);
  L.lw = take(sizeof(float) * MN);
  L.A = take(sizeof(int32_t) * MN);
  L.Cl = take(sizeof(double) * MN);
  L.Sl = take(sizeof(double) * MN);
  L.tile = take(sizeof(double) * (size_t)M * T * pfk::TREC);
  L.mxkey = take(sizeof(uint32_t) * (size_t)M * T);
  L.coff = take(sizeof(double) * (size_t)M * (T + 1));
  L.soff = take(sizeof(double) * (size_t)M * (T + 1));
  L.fstat = take(sizeof(double) * (size_t)M * pfk::FREC);
  // post-resampling partial sums: per tile (T) or per ancestor span (G >= T)
  L.mpart = take(sizeof(double) * (size_t)M * ((N + pfk::ANC_SPAN - 1) / pfk::ANC_SPAN) * dx);
  L.wpart = take(sizeof(double) * (size_t)M * T * dx);
  L.fmean = take(sizeof(double) * (size_t)M * dx);
  L.fmeanw = take(sizeof(double) * (size_t)M * dx);
  L.emean = take(sizeof(double) * 2 * (size_t)dx);
  // grid model: offspring counts and the chunk partial sums of its estimator
  L.cnt = take(grid ? sizeof(int32_t) * MN : 0);
  L.gpart = take(grid ? sizeof(double) * (size_t)M * pfk::grid_est_chunks(N) * 2 * dx : 0);
  L.params = take(learned ? sizeof(float) * (size_t)pfk::mlp_nparams(LEARNED_IN, LEARNED_OUT) : 0);
  L.nearest = take(learned ? sizeof(int32_t) * (size_t)(dx / 2) : 0);
  // ESS schedule: the carried log-weights
  L.lwc = take(carried ? sizeof(float) * MN : 0);
  // auxiliary filter: the pilot log-likelihoods
  L.lpil = take(auxiliary ? sizeof(float) * MN : 0);
  L.end = o;
  return L;
}

// Context-wide arrays after the ensembles: the fused ensemble table, the
// launch plan's tables sized for any tuning (workgroup job lists, at most one
// job per filter per class; batched propagation tiles of the narrowest
// width; the batched grid tables) and the device interval counter.
constexpr int MAX_CLASSES = 40;
constexpr int MIN_PROP_TILE = 64;

struct CtxSizes {
  size_t jobs = 0, tiles = 0, gparticles = 0, gpart_jobs = 0, gfold_jobs = 0;
};

CtxSizes ctx_sizes(const pf_model_desc *models, const pf_ensemble_desc *ens, int n_ens) {
  CtxSizes z;
  for (int e = 0; e < n_ens; ++e) {
    z.jobs += (size_t)ens[e].M;
    z.tiles += (size_t)ens[e].M * (((size_t)ens[e].N + MIN_PROP_TILE - 1) / MIN_PROP_TILE);
    if (models[ens[e].model].kind == PF_MODEL_FHN ||
        models[ens[e].model].kind == PF_MODEL_FHN_PAPER) {
      // room for the padding of the stepping kernel's groups (at most 7)
      z.gparticles += (size_t)ens[e].M * ens[e].N + 7;
      z.gpart_jobs += (size_t)ens[e].M * pfk::grid_est_chunks(ens[e].N);
      z.gfold_jobs += (size_t)ens[e].M;
    }
  }
  return z;
}

size_t ctx_bytes(const pf_model_desc *models, const pf_ensemble_desc *ens, int n_ens) {
  const CtxSizes z = ctx_sizes(models, ens, n_ens);
  return align_up(sizeof(pfk::FusedEns) * (size_t)n_ens) +
         align_up(sizeof(int32_t *) * (size_t)n_ens) +
         MAX_CLASSES * align_up(sizeof(pfk::WgJob) * z.jobs) + 2 * align_up(sizeof(int4) * z.tiles) +
         align_up(sizeof(int4) * z.gparticles) + align_up(sizeof(int4) * z.gpart_jobs) +
         align_up(sizeof(int4) * z.gfold_jobs) + align_up(sizeof(int) * (size_t)n_ens) +
         align_up(sizeof(int));
}

pf_status check_tuning(const pf_tuning &u) {
  if (u.vec_single_kernel != 0 && u.vec_single_kernel != 1)
    return fail(PF_ERR_INVALID_ARG, "vec_single_kernel must be 0 or 1");
  if (u.prop_tile != 64 && u.prop_tile != 128 && u.prop_tile != 256)
    return fail(PF_ERR_INVALID_ARG, "prop_tile must be 64, 128 or 256");
  if (u.resample_bd_min != 64 && u.resample_bd_min != 128 && u.resample_bd_min != 256 &&
      u.resample_bd_min != 512 && u.resample_bd_min != 1024)
    return fail(PF_ERR_INVALID_ARG, "resample_bd_min must be 64, 128, 256, 512 or 1024");
  if (u.grid_blocks_per_cu < 0 || u.grid_blocks_per_cu > 64)
    return fail(PF_ERR_INVALID_ARG, "grid_blocks_per_cu must be in [0, 64]");
  return PF_OK;
}

pf_status check_model(const pf_model_desc &m, int idx) {
  if (m.kind == PF_MODEL_OU1D) {
    if (m.state_dim != 1) return fail(PF_ERR_INVALID_ARG, "model %d: OU needs state_dim 1", idx);
  } else if (m.kind == PF_MODEL_LORENZ63) {
    if (m.state_dim != 3) return fail(PF_ERR_INVALID_ARG, "model %d: Lorenz needs state_dim 3", idx);
  } else if (m.kind == PF_MODEL_FHN) {
    if (m.grid_j < 2 || m.grid_j > 64 || (m.grid_j & 1) || m.state_dim != 2 * m.grid_j * m.grid_j)
      return fail(PF_ERR_INVALID_ARG,
                  "model %d: FH-N needs an even J in [2, 64] and state_dim 2*J*J", idx);
  } else if (m.kind == PF_MODEL_FHN_PAPER) {
    const double l0 = m.params_ext[5];
    if (!(l0 >= 1.0 && l0 <= 32.0) || l0 != std::floor(l0))
      return fail(PF_ERR_INVALID_ARG, "model %d: stimulus duration l0 must be an integer in [1, 32]", idx);
    const int ring = 4 * (((int)l0 + 3) / 4);
    if (m.grid_j < 2 || m.grid_j > 64 || (m.grid_j & 1) ||
        m.state_dim != 2 * m.grid_j * m.grid_j + ring)
      return fail(PF_ERR_INVALID_ARG,
                  "model %d: the FH-N network needs an even J in [2, 64] and state_dim "
                  "2*J*J + %d", idx, ring);
    if (!(m.params_ext[2] >= 0.0 && m.params_ext[2] <= 1.0) || !(m.params_ext[3] < m.params_ext[4]) ||
        !(m.params_ext[6] >= 1.0 && m.params_ext[6] < 2147483647.0) || !(m.params_ext[7] >= 0.0) ||
        !(m.params_ext[6] == std::floor(m.params_ext[6])) ||
        !(m.params_ext[7] == std::floor(m.params_ext[7])))
      return fail(PF_ERR_INVALID_ARG,
                  "model %d: eps in [0, 1], u- < u+, integer forcing period >= 1 and width >= 0", idx);
  } else {
    return fail(PF_ERR_INVALID_ARG, "model %d: unknown kind %d", idx, m.kind);
  }
  if (m.steps_per_obs < 1 || m.steps_per_obs > (1 << 20))
    return fail(PF_ERR_INVALID_ARG, "model %d: steps_per_obs out of range", idx);
  if (!(m.h > 0.0) || !std::isfinite(m.h)) return fail(PF_ERR_INVALID_ARG, "model %d: h <= 0", idx);
  if (m.obs_dim < 1 || m.obs_dim > m.state_dim || !m.h_obs_index)
    return fail(PF_ERR_INVALID_ARG, "model %d: bad obs_dim / obs_index", idx);
  for (int k = 0; k < m.obs_dim; ++k)
    if (m.h_obs_index[k] < 0 || m.h_obs_index[k] >= m.state_dim)
      return fail(PF_ERR_INVALID_ARG, "model %d: obs_index[%d] out of range", idx, k);
  // FH-N: the observation operator reads v (the kernels stage only v for it)
  if (m.kind == PF_MODEL_FHN || m.kind == PF_MODEL_FHN_PAPER)
    for (int k = 0; k < m.obs_dim; ++k)
      if (m.h_obs_index[k] >= m.grid_j * m.grid_j)
        return fail(PF_ERR_INVALID_ARG, "model %d: FH-N obs_index[%d] is not a v node", idx, k);
  if (!(m.obs_var > 0.0) || !std::isfinite(m.obs_var))
    return fail(PF_ERR_INVALID_ARG, "model %d: obs_var must be > 0", idx);
  if (!m.h_prior_mean || !m.h_prior_sd)
    return fail(PF_ERR_INVALID_ARG, "model %d: prior arrays missing", idx);
  for (int k = 0; k < 2; ++k)
    if (!(m.noise_sd[k] >= 0.0)) return fail(PF_ERR_INVALID_ARG, "model %d: noise_sd < 0", idx);
  return PF_OK;
}

pf_status check_all(const pf_model_desc *models, int n_models, const pf_ensemble_desc *ens,
                    int n_ens) {
  if (!models || n_models < 1) return fail(PF_ERR_INVALID_ARG, "no models");
  if (!ens || n_ens < 1) return fail(PF_ERR_INVALID_ARG, "no ensembles");
  for (int i = 0; i < n_models; ++i) PF_TRY(check_model(models[i], i));
  for (int e = 0; e < n_ens; ++e) {
    const pf_ensemble_desc &d = ens[e];
    if (d.model < 0 || d.model >= n_models)
      return fail(PF_ERR_INVALID_ARG, "ensemble %d: model index %d out of range", e, d.model);
    if (d.M < 1 || d.N < 1 || d.N > (1 << 26) || (int64_t)d.M * d.N > (int64_t)1 << 30)
      return fail(PF_ERR_INVALID_ARG, "ensemble %d: bad M=%d N=%d", e, d.M, d.N);
    if (d.M > 65535) return fail(PF_ERR_INVALID_ARG, "ensemble %d: M > 65535", e);
    if (d.flags & ~(PF_ENS_LEARNED | PF_ENS_AUXILIARY))
      return fail(PF_ERR_INVALID_ARG, "ensemble %d: unknown flags 0x%x", e, d.flags);
    if ((d.flags & PF_ENS_AUXILIARY) && ((d.flags & PF_ENS_LEARNED) || d.ess_threshold != 0.0))
      return fail(PF_ERR_UNSUPPORTED,
                  "ensemble %d: the auxiliary filter runs the bootstrap transition and resamples "
                  "at every interval (no PF_ENS_LEARNED, ess_threshold 0)", e);
    if ((d.flags & PF_ENS_LEARNED) &&
        (models[d.model].kind != PF_MODEL_FHN || models[d.model].grid_j > LEARNED_MAX_J))
      return fail(PF_ERR_UNSUPPORTED, "ensemble %d: the learned proposal needs an FH-N model with J <= %d",
                  e, LEARNED_MAX_J);
    if (d.scheme < PF_RESAMPLE_MULTINOMIAL || d.scheme > PF_RESAMPLE_RESIDUAL)
      return fail(PF_ERR_INVALID_ARG, "ensemble %d: unknown resampling scheme %d", e, d.scheme);
    if (d.reserved != 0) return fail(PF_ERR_INVALID_ARG, "ensemble %d: reserved must be 0", e);
    if (!(d.ess_threshold >= 0.0 && d.ess_threshold <= 1.0))
      return fail(PF_ERR_INVALID_ARG, "ensemble %d: ess_threshold must be in [0, 1]", e);
  }
  return PF_OK;
}

// An ensemble with another scheme or an ESS schedule runs on the fused
// path's per-filter resampling kernel only.
bool custom_resampling(const pf_ensemble_desc &d) {
  return d.scheme != PF_RESAMPLE_MULTINOMIAL || d.ess_threshold > 0.0 ||
         (d.flags & PF_ENS_AUXILIARY) != 0;
}

// carried log-weights: the ESS schedule and the auxiliary filter
bool carried_weights(const pf_ensemble_desc &d) {
  return d.ess_threshold > 0.0 || (d.flags & PF_ENS_AUXILIARY) != 0;
}

pf_status check_resampling(const pf_ensemble_desc *ens, int n_ens, uint32_t options) {
  for (int e = 0; e < n_ens; ++e)
    if (custom_resampling(ens[e]) && (!(options & PF_OPT_FUSED) || ens[e].N > pfk::WG_MAX_N))
      return fail(PF_ERR_UNSUPPORTED,
                  "ensemble %d: resampling schemes other than multinomial, the ESS schedule and "
                  "the auxiliary filter need a PF_OPT_FUSED context and N <= %d", e,
                  pfk::WG_MAX_N);
  return PF_OK;
}

pf_status check_fused(const pf_model_desc *models, const pf_ensemble_desc *ens, int n_ens) {
  for (int e = 0; e < n_ens; ++e)
    if ((models[ens[e].model].kind == PF_MODEL_FHN ||
         models[ens[e].model].kind == PF_MODEL_FHN_PAPER) && ens[e].N > pfk::WG_MAX_N)
      return fail(PF_ERR_UNSUPPORTED, "fused path: FH-N ensemble %d has N > %d", e, pfk::WG_MAX_N);
  return PF_OK;
}

size_t total_bytes(const pf_model_desc *models, const pf_ensemble_desc *ens, int n_ens) {
  size_t o = 0;
  for (int e = 0; e < n_ens; ++e) {
    const pf_model_desc &m = models[ens[e].model];
    const int T = (ens[e].N + pfk::TILE - 1) / pfk::TILE;
    o = layout_of(o, ens[e].M, ens[e].N, m.state_dim, m.obs_dim, T,
                  m.kind == PF_MODEL_FHN || m.kind == PF_MODEL_FHN_PAPER,
                  (ens[e].flags & PF_ENS_LEARNED) != 0, carried_weights(ens[e]),
                  (ens[e].flags & PF_ENS_AUXILIARY) != 0)
            .end;
  }
  return o + ctx_bytes(models, ens, n_ens);
}

}  // namespace

struct pf_ctx {
  std::vector<Ens> ens;
  uint32_t options = 0;
  int t = 1;  // interval processed by the next step
  hipStream_t last_stream = nullptr;
  int device = 0;
  // particle buffers, shared by every ensemble: X[cur] holds the particles
  // entering the next interval (to be read through A when `pending`), X[xbar]
  // the pre-resampling particles of the current interval
  int cur = 0, xbar = 1;
  bool pending = false;
  // fused path
  pfk::FusedEns *d_fens = nullptr;
  std::vector<pfk::FusedEns> fz_host;
  std::vector<WgClass> classes;       // workgroup-per-filter launches of every kind
  // staged observations and graph replay
  const float *y_all = nullptr;
  int y_T = 0, dy_total = 0;
  int *d_t = nullptr;  // device interval counter (graph replays)
  bool d_t_valid = false;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int4 *d_tiles[2] = {nullptr, nullptr};  // batched propagation tiles, D = 1 and D = 3
  int n_tiles[2] = {0, 0};
  std::vector<int4> tiles_host[2];
  int32_t **d_counts = nullptr;       // [n_ens] device pointers to offspring counts
  std::vector<int32_t *> counts_host;
  // launch plan of the fused path (pf_tuning) and its tables
  pf_tuning tuning{0, 256, 256, 0};
  int prop_tile = 256;
  pfk::WgJob *d_job_base = nullptr;  // MAX_CLASSES arrays of `max_jobs`
  size_t max_jobs = 0;
  struct GridGroup {
    int J = 0, blocks = 1024;
    std::vector<int4> ptab, part_jobs, fold_jobs;
    std::vector<int> gens;
    int4 *d_ptab = nullptr, *d_part = nullptr, *d_fold = nullptr;
    int *d_gens = nullptr;
  };
  std::vector<GridGroup> ggroups;
  int4 *d_gptab = nullptr, *d_gpart = nullptr, *d_gfold = nullptr;
  int *d_ggens = nullptr;
  // event pairs around the dominant kernel while profiling is enabled
  bool profiling = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_used = 0;
  // second stream of the fused interval: the grid ensembles' chain, forked
  // from and joined to the caller's stream by two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~pf_ctx() {
    for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
    for (int p = 0; p < 2; ++p) {
      if (gexec[p]) (void)hipGraphExecDestroy(gexec[p]);
      if (graph[p]) (void)hipGraphDestroy(graph[p]);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};

namespace {

constexpr size_t MAX_EVENT_PAIRS = 65536;

// Records the start event of a profiled launch; returns the pair index or -1.
long prof_begin(pf_ctx *ctx, hipStream_t s) {
  if (!ctx->profiling || ctx->ev_used >= MAX_EVENT_PAIRS) return -1;
  if (ctx->ev_used == ctx->ev_start.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    ctx->ev_start.push_back(a);
    ctx->ev_stop.push_back(b);
  }
  const size_t i = ctx->ev_used++;
  if (hipEventRecord(ctx->ev_start[i], s) != hipSuccess) return -1;
  return (long)i;
}

void prof_end(pf_ctx *ctx, long i, hipStream_t s) {
  if (i >= 0) (void)hipEventRecord(ctx->ev_stop[(size_t)i], s);
}

// gather x' = xbar[A] of one ensemble from buffer `from` into buffer `to`
hipError_t gather(const Ens &E, int from, int to, hipStream_t s) {
  const pfk::EnsDev &D = E.dev;
  return E.grid ? pfk::launch_grid_gather(D, D.X[from], D.X[to], s)
                : pfk::launch_vec_gather(D, D.X[from], D.X[to], s);
}

// offset of ensemble E's observations in the concatenated observation vector
int learned_yoff(const pf_ctx *ctx, const Ens &E) {
  int o = 0;
  for (const Ens &F : ctx->ens) {
    if (&F == &E) break;
    o += F.dy;
  }
  return o;
}

pf_status stage_run(pf_ctx *ctx, uint32_t stages, const float *d_y, hipStream_t s) {
  const int t = ctx->t;
  if ((stages & PF_STAGE_WEIGHT) && !d_y)
    return fail(PF_ERR_INVALID_ARG, "weighting needs observations");
  if (stages & PF_STAGE_PROPAGATE) {
    const int out = 1 - ctx->cur;
    for (size_t e = 0; e < ctx->ens.size(); ++e) {
      Ens &E = ctx->ens[e];
      pfk::EnsDev &D = E.dev;
      const int32_t *anc = ctx->pending ? D.A : nullptr;
      if (E.paper) {
        const long ev = prof_begin(ctx, s);
        PF_HIP(pfk::launch_fhnp_steps(ctx->d_fens, (int)e, E.d.M, E.d.N, D.md.J,
                                      pfk::IvArg{t, nullptr, nullptr, 0}, ctx->cur,
                                      ctx->pending ? 1 : 0, s));
        prof_end(ctx, ev, s);
      } else if (E.learned) {
        if (!d_y) return fail(PF_ERR_INVALID_ARG, "the learned proposal needs the observations");
        const long ev = prof_begin(ctx, s);
        PF_HIP(pfk::launch_grid_steps_learned(D, pfk::IvArg{t, nullptr, d_y, 0}, learned_yoff(ctx, E),
                                              D.X[ctx->cur], anc, D.X[out], D.lw, E.params,
                                              E.nearest, E.sd0, E.sd1, E.lblocks, s));
        prof_end(ctx, ev, s);
      } else if (!E.grid) {
        const long ev = prof_begin(ctx, s);
        PF_HIP(pfk::launch_vec_propagate(D, t, D.X[ctx->cur], anc, D.X[out], nullptr, nullptr, s));
        prof_end(ctx, ev, s);
      } else {
        // one streaming launch per Euler step: the first reads through the
        // ancestors into the other buffer, the rest update it in place
        for (int st = 0; st < D.md.S; ++st) {
          const long ev = prof_begin(ctx, s);
          PF_HIP(pfk::launch_grid_stream_step(D, (t - 1) * D.md.S + st,
                                              st == 0 ? D.X[ctx->cur] : D.X[out],
                                              st == 0 ? anc : nullptr, D.X[out], nullptr, nullptr,
                                              E.blocks, s));
          prof_end(ctx, ev, s);
        }
      }
    }
    ctx->xbar = out;
    ctx->pending = false;
  }
  size_t yoff = 0;
  for (Ens &E : ctx->ens) {
    pfk::EnsDev &D = E.dev;
    const float *y = d_y ? d_y + yoff : nullptr;
    yoff += (size_t)E.dy;
    if ((stages & PF_STAGE_WEIGHT) && !E.learned) {
      if (E.grid)
        PF_HIP(pfk::launch_grid_loglik(D, D.X[ctx->xbar], y, s));
      else
        PF_HIP(pfk::launch_vec_loglik(D, D.X[ctx->xbar], y, s));
    }
    if (stages & PF_STAGE_RESAMPLE) PF_HIP(pfk::launch_resample(D, t, s));
    if (stages & PF_STAGE_GATHER) PF_HIP(gather(E, ctx->xbar, 1 - ctx->xbar, s));
  }
  if (stages & PF_STAGE_GATHER) {
    ctx->cur = 1 - ctx->xbar;
    ctx->pending = false;
  }
  if (stages & PF_STAGE_ESTIMATE) {
    for (Ens &E : ctx->ens) {
      pfk::EnsDev &D = E.dev;
      if (E.grid) {
        // sum_i n_i xbar_i / N with the offspring counts n_i of the ancestors
        PF_HIP(pfk::launch_offspring_counts(D, E.cnt, s));
        PF_HIP(pfk::launch_grid_estimate(D, D.X[ctx->xbar], E.cnt, E.gpart, s));
      } else {
        if (ctx->pending) return fail(PF_ERR_STATE, "estimate stage needs gathered particles");
        PF_HIP(pfk::launch_vec_estimate(D, D.X[ctx->cur], D.X[ctx->xbar], nullptr, true, s));
      }
    }
  }
  ctx->last_stream = s;
  return PF_OK;
}

// The fused interval: one filter-per-workgroup launch per class, the tiled
// kernels for ensembles whose filters exceed one workgroup, and the
// cross-filter averages.  The particles stay where propagation wrote them
// and the next interval gathers them through the ancestors.
// The two chains of a fused interval share no data until the cross-filter
// means: the vector ensembles' (propagation tiles, single-kernel filters,
// resampling with their estimates) and the grid ensembles' (stepping,
// learned stepping, resampling, state-wide estimators).  When a batch holds
// both, the grid chain runs on a second stream (default priority) forked
// from the caller's stream and joined back before the means, so that one
// chain's latency-bound launches overlap the other's compute; in a captured
// graph the fork and join become dependencies.  While profiling, both run
// in order on the caller's stream, so that the timed kernels do not share
// the device.
pf_status side_stream(pf_ctx *ctx) {
  if (!ctx->side) PF_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  if (!ctx->ev_fork) PF_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  if (!ctx->ev_join) PF_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  return PF_OK;
}

pf_status fused_launch(pf_ctx *ctx, pfk::IvArg iv, int parity, int pending, bool resample_only,
                       hipStream_t s) {
  const int out = 1 - parity;  // buffer that holds xbar of this interval
  const bool prof = !ctx->capturing && !resample_only;
  bool vec_work = ctx->n_tiles[0] + ctx->n_tiles[1] > 0, grid_work = !ctx->ggroups.empty();
  for (const WgClass &c : ctx->classes) {
    if (c.kind == CLASS_FILTER_WG || c.kind == CLASS_RESAMPLE_VEC) vec_work = true;
    if (c.kind == CLASS_RESAMPLE_GRID) grid_work = true;
  }
  for (const Ens &E : ctx->ens) {
    if (E.learned || E.paper) grid_work = true;
    else if (E.tiled) vec_work = true;
  }
  hipStream_t g = s;  // the grid chain's stream
  if (vec_work && grid_work && !resample_only && !ctx->profiling) {
    PF_TRY(side_stream(ctx));
    PF_HIP(hipEventRecord(ctx->ev_fork, s));
    PF_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    g = ctx->side;
  }
  // 0. auxiliary filters: the pilot of every particle and the first-stage
  //    resampling from its weights (the grid ensembles' on the grid chain)
  if (!resample_only) {
    for (size_t e = 0; e < ctx->ens.size(); ++e) {
      const Ens &E = ctx->ens[e];
      if (!E.apf) continue;
      if (E.paper)
        PF_HIP(pfk::launch_fhnp_pilot(ctx->d_fens, (int)e, E.d.M, E.d.N, E.dev.md.J, iv, parity,
                                      pending, g));
      else if (E.grid)
        PF_HIP(pfk::launch_grid_pilot(ctx->d_fens, (int)e, E.d.M, E.d.N, E.dev.md.J, iv, parity,
                                      pending, g));
      else
        PF_HIP(pfk::launch_vec_pilot(E.dx, ctx->d_fens, (int)e, E.d.M, E.d.N, iv, parity, pending,
                                     s));
    }
    for (const WgClass &c : ctx->classes)
      if (c.kind == CLASS_APF_FIRST)
        PF_HIP(pfk::launch_resample_wg(c.D, c.BD, c.d_jobs, (int)c.jobs.size(), c.max_n,
                                       ctx->d_fens, iv, ctx->d_counts, parity, true, 1,
                                       c.D == 0 ? g : s));
  }
  // 1. propagation + weighting: the batched vector tiles (profiled: the
  //    kernel that carries the interval), the single-kernel classes, and the
  //    grid model's stepping kernel (profiled)
  if (!resample_only) {
    const long ev = (prof && ctx->n_tiles[0] + ctx->n_tiles[1]) ? prof_begin(ctx, s) : -1;
    for (int w = 1; w >= 0; --w)
      PF_HIP(pfk::launch_vec_prop_batched(w ? 3 : 1, ctx->d_tiles[w], ctx->n_tiles[w],
                                          ctx->prop_tile, ctx->d_fens, iv, parity, pending, s));
    prof_end(ctx, ev, s);
  }
  for (const WgClass &c : ctx->classes)
    if (c.kind == CLASS_FILTER_WG) {
      const long ev = prof ? prof_begin(ctx, s) : -1;
      PF_HIP(pfk::launch_filter_wg(c.D, c.BD, c.d_jobs, (int)c.jobs.size(), c.max_n, ctx->d_fens,
                                   iv, parity, pending, resample_only ? 1 : 0, s));
      prof_end(ctx, ev, s);
    }
  if (!resample_only) {
    // every bootstrap grid ensemble of one grid size in one launch (profiled)
    for (const auto &gg : ctx->ggroups) {
      const long eg = prof ? prof_begin(ctx, g) : -1;
      PF_HIP(pfk::launch_grid_steps_batched(gg.J, gg.d_ptab, (int)gg.ptab.size(), ctx->d_fens, iv,
                                            parity, pending, gg.blocks, g));
      prof_end(ctx, eg, g);
    }
    for (size_t e = 0; e < ctx->ens.size(); ++e) {
      const Ens &E = ctx->ens[e];
      if (!E.paper) continue;
      const long eg = prof ? prof_begin(ctx, g) : -1;
      PF_HIP(pfk::launch_fhnp_steps(ctx->d_fens, (int)e, E.d.M, E.d.N, E.dev.md.J, iv, parity,
                                    pending, g));
      prof_end(ctx, eg, g);
    }
    int yo = 0;
    for (Ens &E : ctx->ens) {
      const int yoff = yo;
      yo += E.dy;
      if (!E.learned) continue;
      pfk::EnsDev &D = E.dev;
      const long eg = prof ? prof_begin(ctx, g) : -1;
      PF_HIP(pfk::launch_grid_steps_learned(D, iv, yoff, D.X[parity], pending ? D.A : nullptr,
                                            D.X[out], D.lw, E.params, E.nearest, E.sd0, E.sd1,
                                            E.lblocks, g));
      prof_end(ctx, eg, g);
    }
  }
  // 2. resampling and the filters' estimates
  for (const WgClass &c : ctx->classes) {
    if (c.kind == CLASS_RESAMPLE_VEC)
      PF_HIP(pfk::launch_resample_wg(c.D, c.BD, c.d_jobs, (int)c.jobs.size(), c.max_n, ctx->d_fens,
                                     iv, ctx->d_counts, out, c.custom, 0, s));
    else if (c.kind == CLASS_RESAMPLE_GRID)
      PF_HIP(pfk::launch_resample_wg(0, c.BD, c.d_jobs, (int)c.jobs.size(), c.max_n, ctx->d_fens,
                                     iv, ctx->d_counts, out, c.custom, 0, g));
  }
  for (const auto &gg : ctx->ggroups)
    PF_HIP(pfk::launch_grid_estimate_batched(gg.J, gg.d_part, (int)gg.part_jobs.size(), gg.d_fold,
                                             (int)gg.fold_jobs.size(), gg.d_gens, (int)gg.gens.size(),
                                             ctx->d_fens, out, g));
  for (Ens &E : ctx->ens) {
    pfk::EnsDev &D = E.dev;
    if (E.learned || E.paper) {
      PF_HIP(pfk::launch_grid_estimate(D, D.X[out], E.cnt, E.gpart, g));
    } else if (E.tiled && E.fz.mpart) {
      // (in a resampling-only interval no propagation has raised the keys)
      PF_HIP(pfk::launch_resample_fused(D, iv, D.X[out], !resample_only, s));
    } else if (E.tiled) {
      PF_HIP(pfk::launch_resample(D, iv.t, s, iv.tp));
      PF_HIP(pfk::launch_vec_estimate(D, D.X[out], D.X[out], D.A, false, s));
    }
  }
  if (g != s) {
    PF_HIP(hipEventRecord(ctx->ev_join, g));
    PF_HIP(hipStreamWaitEvent(s, ctx->ev_join, 0));
  }
  // 3. the cross-filter averages (and, in a graph, the interval counter);
  //    grid ensembles have theirs from their own estimator, so a batch of
  //    grid ensembles only needs the launch for the counter
  int max_m = 1;
  bool any_vec = false, any_tiled = false;
  for (const Ens &E : ctx->ens) {
    max_m = std::max(max_m, (int)E.d.M);
    any_vec |= !E.grid;
    // (four waves fold up to four tiled filters in one round; more take 16)
    any_tiled |= E.tiled && E.fz.mpart != nullptr && E.d.M > 4;
  }
  if (any_vec || iv.tp)
    PF_HIP(pfk::launch_ensemble_means(ctx->d_fens, (int)ctx->ens.size(), max_m, any_tiled,
                                      iv.tp ? const_cast<int *>(iv.tp) : nullptr, s));
  return PF_OK;
}

// The fused interval launched directly.
pf_status fused_run(pf_ctx *ctx, const float *d_y, hipStream_t s, bool resample_only) {
  const int parity = resample_only ? 1 - ctx->xbar : ctx->cur;
  const int pending = (!resample_only && ctx->pending) ? 1 : 0;
  const pfk::IvArg iv{ctx->t, nullptr, d_y, 0};
  PF_TRY(fused_launch(ctx, iv, parity, pending, resample_only, s));
  if (resample_only) {
    ctx->cur = ctx->xbar;
  } else {
    ctx->cur = 1 - ctx->cur;
    ctx->xbar = ctx->cur;
  }
  ctx->pending = true;
  ctx->last_stream = s;
  return PF_OK;
}

// The fused interval replayed from a captured graph (one graph per buffer
// parity; interval index and observations come from device memory).
pf_status graph_step(pf_ctx *ctx, hipStream_t s) {
  const int parity = ctx->cur;
  if (!ctx->gexec[parity]) {
    if (!ctx->cap_stream) PF_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const pfk::IvArg iv{0, ctx->d_t, ctx->y_all, ctx->dy_total};
    PF_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    const pf_status st = fused_launch(ctx, iv, parity, 1, false, ctx->cap_stream);
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
    if (st != PF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    PF_HIP(ce);
    ctx->graph[parity] = g;
    PF_HIP(hipGraphInstantiate(&ctx->gexec[parity], g, nullptr, nullptr, 0));
  }
  if (!ctx->d_t_valid) {
    PF_HIP(pfk::launch_set_i32(ctx->d_t, ctx->t, s));
    ctx->d_t_valid = true;
  }
  const long ev = prof_begin(ctx, s);
  PF_HIP(hipGraphLaunch(ctx->gexec[parity], s));
  prof_end(ctx, ev, s);
  ctx->cur = 1 - ctx->cur;
  ctx->xbar = ctx->cur;
  ctx->pending = true;
  ctx->last_stream = s;
  return PF_OK;
}

void drop_graphs(pf_ctx *ctx) {
  for (int p = 0; p < 2; ++p) {
    if (ctx->gexec[p]) (void)hipGraphExecDestroy(ctx->gexec[p]);
    if (ctx->graph[p]) (void)hipGraphDestroy(ctx->graph[p]);
    ctx->gexec[p] = nullptr;
    ctx->graph[p] = nullptr;
  }
}

// Resolve pending ancestors: gather every ensemble into the other buffer.
pf_status materialise(pf_ctx *ctx, hipStream_t s) {
  if (!ctx->pending) return PF_OK;
  for (Ens &E : ctx->ens) PF_HIP(gather(E, ctx->cur, 1 - ctx->cur, s));
  ctx->xbar = ctx->cur;
  ctx->cur = 1 - ctx->cur;
  ctx->pending = false;
  return PF_OK;
}

// The launch plan of the fused path for a tuning: which vector ensembles run
// in the single filter-per-workgroup kernel, the workgroup-per-filter classes
// (by kind, state dimension and workgroup size, filters of larger N first),
// the batched propagation tiles, and the batched grid tables (per grid size
// J; ensembles with the learned proposal keep their own launch).  The tables
// live at fixed offsets sized for any tuning; the caller has made sure no
// work still reads them.
pf_status build_plan(pf_ctx *ctx, const pf_tuning &u, hipStream_t s) {
  PF_TRY(check_tuning(u));
  const int n_ens = (int)ctx->ens.size();
  // (the single-kernel path resamples multinomially at every interval)
  for (Ens &E : ctx->ens)
    E.wg = !E.grid && E.d.N <= pfk::WG_MAX_N && u.vec_single_kernel && !custom_resampling(E.d);
  ctx->classes.clear();
  int next_class = 0;
  const int BDs[5] = {1024, 512, 256, 128, 64};
  auto add_class = [&](int kind, int D, int BD, int bd_min, bool custom, auto member) {
    WgClass c;
    c.kind = kind;
    c.D = D;
    c.BD = BD;
    c.custom = custom;
    c.max_n = 0;
    std::vector<std::pair<int, int>> order;  // (N, ensemble)
    for (int e = 0; e < n_ens; ++e) {
      const Ens &E = ctx->ens[(size_t)e];
      if (member(E) && custom_resampling(E.d) == custom && wg_block(E.d.N, bd_min) == BD)
        order.push_back({E.d.N, e});
    }
    if (order.empty()) return;
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
                       return a.first > b.first;
                     });
    for (auto &pr : order) {
      c.max_n = std::max(c.max_n, pr.first);
      for (int mm = 0; mm < ctx->ens[(size_t)pr.second].d.M; ++mm)
        c.jobs.push_back(pfk::WgJob{pr.second, mm});
    }
    c.d_jobs = ctx->d_job_base + (size_t)next_class++ * (align_up(sizeof(pfk::WgJob) * ctx->max_jobs) /
                                                        sizeof(pfk::WgJob));
    ctx->classes.push_back(std::move(c));
  };
  // the single-kernel path holds one element per thread below 1024 threads
  const int wg_min = std::max(256, u.resample_bd_min);
  for (int D : {3, 1}) {
    for (int BD : BDs) {
      if (BD >= 256)
        add_class(CLASS_FILTER_WG, D, BD, wg_min, false,
                  [D](const Ens &E) { return E.wg && E.dx == D; });
      for (bool custom : {false, true})
        add_class(CLASS_RESAMPLE_VEC, D, BD, u.resample_bd_min, custom, [D](const Ens &E) {
          return !E.grid && !E.wg && !E.tiled && E.dx == D;
        });
    }
  }
  for (int BD : BDs)
    for (bool custom : {false, true})
      add_class(CLASS_RESAMPLE_GRID, 0, BD, u.resample_bd_min, custom,
                [](const Ens &E) { return E.grid && E.d.N <= pfk::WG_MAX_N; });
  // the first-stage resampling of auxiliary filters (its estimates are
  // overwritten by the second stage's)
  for (int D : {3, 1, 0})
    for (int BD : BDs)
      add_class(CLASS_APF_FIRST, D, BD, u.resample_bd_min, true, [D](const Ens &E) {
        return E.apf && (E.grid ? 0 : E.dx) == D;
      });
  if (next_class > MAX_CLASSES) return fail(PF_ERR_STATE, "too many launch classes");
  // batched propagation tiles of the vector ensembles not run by the single
  // filter-per-workgroup kernel
  ctx->prop_tile = u.prop_tile;
  for (int w = 0; w < 2; ++w) ctx->tiles_host[w].clear();
  {
    // Workgroups of a launch go to the 8 XCDs in turn (workgroup b to XCD
    // b mod 8), and each XCD has its own L2.  A filter resampled by
    // workgroup j of its class runs there on XCD j mod 8; its propagation
    // tiles are placed on the positions of that same XCD, so that the
    // resampler's reads of the log-weights and predicted states and the
    // next interval's reads through the ancestors find the lines in the L2
    // that wrote them.  (Any order is correct; this one is the locality.)
    constexpr int XCDS = 8;
    std::vector<std::vector<int>> xpos((size_t)n_ens);
    for (int e = 0; e < n_ens; ++e) xpos[(size_t)e].assign((size_t)ctx->ens[(size_t)e].d.M, -1);
    for (const WgClass &c : ctx->classes)
      if (c.kind == CLASS_RESAMPLE_VEC)
        for (size_t j = 0; j < c.jobs.size(); ++j)
          xpos[(size_t)c.jobs[j].ens][(size_t)c.jobs[j].filter] = (int)(j % XCDS);
    auto xcd = [&](int e, int mm) {
      const int x = xpos[(size_t)e][(size_t)mm];
      return x >= 0 ? x : mm % XCDS;
    };
    std::vector<int4> bucket[2][XCDS];
    for (int e = 0; e < n_ens; ++e) {
      const Ens &E = ctx->ens[(size_t)e];
      if (E.grid || E.wg) continue;
      const int which = E.dx == 3 ? 1 : 0;
      for (int mm = 0; mm < E.d.M; ++mm)
        for (int i0 = 0; i0 < E.d.N; i0 += u.prop_tile) {
          // a tiled ensemble: resampling tile q of filter m is workgroup
          // q + T m of its CDF launch, so the propagation tiles of its
          // particles go to that workgroup's XCD
          const int x = E.tiled ? (int)(((long)(i0 / pfk::TILE) + (long)E.T * mm) % XCDS)
                                : xcd(e, mm);
          bucket[which][x].push_back(int4{e, mm, i0, 0});
        }
    }
    for (int w = 0; w < 2; ++w) {
      size_t total = 0, next[XCDS] = {};
      for (int x = 0; x < XCDS; ++x) total += bucket[w][x].size();
      for (size_t b = 0; b < total; ++b) {
        // position b's own XCD while it has tiles, else the fullest other
        int x = (int)(b % XCDS);
        if (next[x] == bucket[w][x].size()) {
          size_t most = 0;
          for (int q = 0; q < XCDS; ++q)
            if (bucket[w][q].size() - next[q] > most) {
              most = bucket[w][q].size() - next[q];
              x = q;
            }
        }
        ctx->tiles_host[w].push_back(bucket[w][x][next[x]++]);
      }
    }
  }
  for (int w = 0; w < 2; ++w) ctx->n_tiles[w] = (int)ctx->tiles_host[w].size();
  // batched grid tables, one group per grid size
  ctx->ggroups.clear();
  size_t op = 0, oj = 0, of = 0, og = 0;
  for (int e = 0; e < n_ens; ++e) {
    const Ens &E = ctx->ens[(size_t)e];
    if (!E.grid || E.learned || E.paper) continue;
    const int J = E.dev.md.J;
    pf_ctx::GridGroup *g = nullptr;
    for (auto &gg : ctx->ggroups)
      if (gg.J == J) g = &gg;
    if (!g) {
      ctx->ggroups.emplace_back();
      g = &ctx->ggroups.back();
      g->J = J;
    }
    const int nch = pfk::grid_est_chunks(E.d.N);
    for (int mm = 0; mm < E.d.M; ++mm) {
      for (int i = 0; i < E.d.N; ++i) g->ptab.push_back(int4{e, mm, i, 0});
      for (int ch = 0; ch < nch; ++ch) g->part_jobs.push_back(int4{e, mm, ch, 0});
      g->fold_jobs.push_back(int4{e, mm, 0, 0});
    }
    // the stepping kernel takes ppb entries of one ensemble per workgroup
    const size_t ppb = (size_t)pfk::grid_steps_ppb(J);
    while (g->ptab.size() % ppb) g->ptab.push_back(int4{-1, 0, 0, 0});
    g->gens.push_back(e);
  }
  for (auto &g : ctx->ggroups) {
    const int occ = pfk::grid_resident_blocks_j(g.J);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    g.blocks = u.grid_blocks_per_cu > 0 ? std::min(occ, u.grid_blocks_per_cu * cus) : occ;
    g.d_ptab = ctx->d_gptab + op;
    g.d_part = ctx->d_gpart + oj;
    g.d_fold = ctx->d_gfold + of;
    g.d_gens = ctx->d_ggens + og;
    op += g.ptab.size();
    oj += g.part_jobs.size();
    of += g.fold_jobs.size();
    og += g.gens.size();
  }
  // upload
  for (WgClass &c : ctx->classes)
    PF_HIP(hipMemcpyAsync(c.d_jobs, c.jobs.data(), sizeof(pfk::WgJob) * c.jobs.size(),
                          hipMemcpyHostToDevice, s));
  for (int w = 0; w < 2; ++w)
    if (ctx->n_tiles[w] > 0)
      PF_HIP(hipMemcpyAsync(ctx->d_tiles[w], ctx->tiles_host[w].data(),
                            sizeof(int4) * ctx->tiles_host[w].size(), hipMemcpyHostToDevice, s));
  for (auto &g : ctx->ggroups) {
    PF_HIP(hipMemcpyAsync(g.d_ptab, g.ptab.data(), sizeof(int4) * g.ptab.size(),
                          hipMemcpyHostToDevice, s));
    PF_HIP(hipMemcpyAsync(g.d_part, g.part_jobs.data(), sizeof(int4) * g.part_jobs.size(),
                          hipMemcpyHostToDevice, s));
    PF_HIP(hipMemcpyAsync(g.d_fold, g.fold_jobs.data(), sizeof(int4) * g.fold_jobs.size(),
                          hipMemcpyHostToDevice, s));
    PF_HIP(hipMemcpyAsync(g.d_gens, g.gens.data(), sizeof(int) * g.gens.size(),
                          hipMemcpyHostToDevice, s));
  }
  // the host tables are kept in the context, so the copies may stay queued;
  // captured graphs refer to the old plan
  drop_graphs(ctx);
  ctx->tuning = u;
  return PF_OK;
}

// Every filter back to its prior draw and interval 1 (log-evidence and
// statistics cleared), as after pf_init.
pf_status reset_filters(pf_ctx *ctx, hipStream_t s) {
  for (Ens &E : ctx->ens) {
    pfk::EnsDev &D = E.dev;
    PF_HIP(hipMemsetAsync(D.fstat, 0, sizeof(double) * (size_t)E.d.M * pfk::FREC, s));
    PF_HIP(hipMemsetAsync(D.emean, 0, sizeof(double) * 2 * (size_t)E.dx, s));
    PF_HIP(hipMemsetAsync(D.A, 0, sizeof(int32_t) * (size_t)E.d.M * E.d.N, s));
    if (E.lwc) PF_HIP(pfk::launch_fill_f32(E.lwc, 0.f, (size_t)E.d.M * E.d.N, s));
    if (E.grid)
      PF_HIP(pfk::launch_grid_init(D, D.X[0], s));
    else
      PF_HIP(pfk::launch_vec_init(D, D.X[0], s));
  }
  ctx->cur = 0;
  ctx->xbar = 1;
  ctx->pending = false;
  ctx->t = 1;
  ctx->d_t_valid = false;
  return PF_OK;
}

Ens *get_ens(pf_ctx *ctx, int32_t e) {
  if (!ctx || e < 0 || e >= (int32_t)ctx->ens.size()) return nullptr;
  return &ctx->ens[(size_t)e];
}

}  // namespace

extern "C" {

pf_status pf_workspace_bytes(const pf_model_desc *h_models, int32_t n_models,
                             const pf_ensemble_desc *h_ens, int32_t n_ens, uint32_t options,
                             size_t *out_bytes) {
  if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
  if (options > (PF_OPT_FUSED | PF_OPT_GRAPH)) return fail(PF_ERR_INVALID_ARG, "unknown options");
  PF_TRY(check_all(h_models, n_models, h_ens, n_ens));
  if (options & PF_OPT_FUSED) PF_TRY(check_fused(h_models, h_ens, n_ens));
  PF_TRY(check_resampling(h_ens, n_ens, options));
  *out_bytes = total_bytes(h_models, h_ens, n_ens);
  return PF_OK;
}

pf_status pf_init(const pf_model_desc *h_models, int32_t n_models, const pf_ensemble_desc *h_ens,
                  int32_t n_ens, uint32_t options, void *d_workspace, size_t workspace_bytes,
                  void *stream, pf_ctx **out_ctx) {
  if (!out_ctx) return fail(PF_ERR_INVALID_ARG, "out_ctx is NULL");
  *out_ctx = nullptr;
  if (options > (PF_OPT_FUSED | PF_OPT_GRAPH)) return fail(PF_ERR_INVALID_ARG, "unknown options");
  if ((options & PF_OPT_GRAPH) && !(options & PF_OPT_FUSED))
    return fail(PF_ERR_INVALID_ARG, "PF_OPT_GRAPH needs PF_OPT_FUSED");
  PF_TRY(check_all(h_models, n_models, h_ens, n_ens));
  if (options & PF_OPT_FUSED) PF_TRY(check_fused(h_models, h_ens, n_ens));
  PF_TRY(check_resampling(h_ens, n_ens, options));
  const size_t need = total_bytes(h_models, h_ens, n_ens);
  if (!d_workspace || ((uintptr_t)d_workspace % ALIGN) != 0)
    return fail(PF_ERR_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  if (workspace_bytes < need)
    return fail(PF_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, need);

  hipStream_t s = (hipStream_t)stream;
  int device = 0;
  PF_HIP(hipGetDevice(&device));
  pf_ctx *ctx = new pf_ctx();
  ctx->options = options;
  ctx->device = device;
  char *ws = (char *)d_workspace;
  size_t base = 0, yoff_acc = 0;
  ctx->ens.resize((size_t)n_ens);
  for (int e = 0; e < n_ens; ++e) {
    Ens &E = ctx->ens[(size_t)e];
    E.d = h_ens[e];
    const pf_model_desc &m = h_models[E.d.model];
    E.dx = m.state_dim;
    E.dy = m.obs_dim;
    E.grid = m.kind == PF_MODEL_FHN || m.kind == PF_MODEL_FHN_PAPER;
    E.paper = m.kind == PF_MODEL_FHN_PAPER;
    E.T = (E.d.N + pfk::TILE - 1) / pfk::TILE;
    E.obs_idx.assign(m.h_obs_index, m.h_obs_index + m.obs_dim);
    E.prior_mean.resize((size_t)E.dx);
    E.prior_sd.resize((size_t)E.dx);
    for (int k = 0; k < E.dx; ++k) {
      E.prior_mean[(size_t)k] = (float)m.h_prior_mean[k];
      E.prior_sd[(size_t)k] = (float)m.h_prior_sd[k];
    }
    E.learned = (E.d.flags & PF_ENS_LEARNED) != 0;
    E.apf = (E.d.flags & PF_ENS_AUXILIARY) != 0;
    const Layout L = layout_of(base, E.d.M, E.d.N, E.dx, E.dy, E.T, E.grid, E.learned,
                               carried_weights(E.d), E.apf);
    base = L.end;
    pfk::EnsDev &D = E.dev;
    pfk::ModelDev &md = D.md;
    md.kind = m.kind;
    md.dx = E.dx;
    md.J = m.grid_j;
    md.S = m.steps_per_obs;
    md.dy = E.dy;
    md.h = (float)m.h;
    md.p0 = (float)m.params[0];
    md.p1 = (float)m.params[1];
    md.p2 = (float)m.params[2];
    md.p3 = (float)m.params[3];
    md.sq0 = (float)(m.noise_sd[0] * std::sqrt(m.h));
    md.sq1 = (float)(m.noise_sd[1] * std::sqrt(m.h));
    md.inv2var = (float)(1.0 / (2.0 * m.obs_var));
    md.stim_b2 = (float)m.params_ext[0];
    md.stim_amp = (float)m.params_ext[1];
    md.stim_eps = m.params_ext[2];
    md.stim_lo = (float)m.params_ext[3];
    md.stim_hi = (float)m.params_ext[4];
    md.stim_l0 = (int32_t)m.params_ext[5];
    md.force_period = E.paper ? (int32_t)m.params_ext[6] : 1;
    md.force_width = (int32_t)m.params_ext[7];
    md.obs_sd = (float)std::sqrt(m.obs_var);
    md.obs_idx = (const int32_t *)(ws + L.obs);
    md.prior_mean = (const float *)(ws + L.pmean);
    md.prior_sd = (const float *)(ws + L.psd);
    D.key = pfk::make_key(E.d.seed);
    D.M = E.d.M;
    D.N = E.d.N;
    D.T = E.T;
    D.lognorm = -0.5 * m.obs_dim * std::log(2.0 * M_PI * m.obs_var);
    D.X[0] = (float *)(ws + L.X0);
    D.X[1] = (float *)(ws + L.X1);
    D.lw = (float *)(ws + L.lw);
    D.A = (int32_t *)(ws + L.A);
    D.Cl = (double *)(ws + L.Cl);
    D.Sl = (double *)(ws + L.Sl);
    D.tile = (double *)(ws + L.tile);
    D.mxkey = (uint32_t *)(ws + L.mxkey);
    D.coff = (double *)(ws + L.coff);
    D.soff = (double *)(ws + L.soff);
    D.fstat = (double *)(ws + L.fstat);
    D.mpart = (double *)(ws + L.mpart);
    D.wpart = (double *)(ws + L.wpart);
    D.fmean = (double *)(ws + L.fmean);
    D.fmeanw = (double *)(ws + L.fmeanw);
    D.emean = (double *)(ws + L.emean);
    // fused-path record
    pfk::FusedEns &F = E.fz;
    F.md = md;
    F.key = D.key;
    F.M = E.d.M;
    F.N = E.d.N;
    F.yoff = (int32_t)yoff_acc;
    yoff_acc += (size_t)E.dy;
    F.lognorm = D.lognorm;
    F.X0 = D.X[0];
    F.X1 = D.X[1];
    F.lw = D.lw;
    F.A = D.A;
    F.fstat = D.fstat;
    F.fmean = D.fmean;
    F.fmeanw = D.fmeanw;
    F.emean = D.emean;
    E.wg = false;  // set by the launch plan
    E.tiled = !E.grid && E.d.N > pfk::WG_MAX_N;
    // tiled filters on the fused path: propagation raises the tile maximum
    // keys; up to FOLD_MAX_TILES tiles the resampler folds the tile offsets
    // and the cross-filter means fold the estimator's partial sums
    F.T = E.T;
    F.G = (E.d.N + pfk::ANC_SPAN - 1) / pfk::ANC_SPAN;
    F.mxkey = E.tiled ? D.mxkey : nullptr;
    const bool fold = E.tiled && E.T <= pfk::FOLD_MAX_TILES;
    F.mpart = fold ? D.mpart : nullptr;
    F.wpart = fold ? D.wpart : nullptr;
    F.cnt = nullptr;
    F.gpart = nullptr;
    F.nch = 0;
    F.scheme = E.d.scheme;
    F.ess_thr = E.d.ess_threshold;
    F.lwc = carried_weights(E.d) ? (float *)(ws + L.lwc) : nullptr;
    E.lwc = F.lwc;
    F.apf = E.apf ? 1 : 0;
    F.lpil = E.apf ? (float *)(ws + L.lpil) : nullptr;
    if (E.grid) {
      E.cnt = (int32_t *)(ws + L.cnt);
      E.gpart = (double *)(ws + L.gpart);
      E.blocks = pfk::grid_resident_blocks(md);
      F.cnt = E.cnt;
      F.gpart = E.gpart;
      F.nch = pfk::grid_est_chunks(E.d.N);
    }
    std::vector<int32_t> near_host;
    if (E.learned) {
      E.params = (float *)(ws + L.params);
      E.nearest = (int32_t *)(ws + L.nearest);
      E.sd0 = m.noise_sd[0];
      E.sd1 = m.noise_sd[1];
      E.lblocks = pfk::learned_resident_blocks(md.J);
      // nearest observed node of every node: least squared distance on the
      // grid, ties to the lower observation index
      const int J = md.J;
      near_host.resize((size_t)J * J);
      for (int n = 0; n < J * J; ++n) {
        const int i = n / J, j = n % J;
        long best = -1;
        for (int o = 0; o < E.dy; ++o) {
          const int r = E.obs_idx[(size_t)o] / J, c = E.obs_idx[(size_t)o] % J;
          const long d2 = (long)(i - r) * (i - r) + (long)(j - c) * (j - c);
          if (best < 0 || d2 < best) {
            best = d2;
            near_host[(size_t)n] = o;
          }
        }
      }
    }
    pf_status st = PF_OK;
#define INIT_TRY(expr)                                  \
  do {                                                  \
    st = dev((expr), #expr);                            \
    if (st != PF_OK) {                                  \
      delete ctx;                                       \
      return st;                                        \
    }                                                   \
  } while (0)
    INIT_TRY(hipMemcpyAsync((void *)md.obs_idx, E.obs_idx.data(), sizeof(int32_t) * E.dy,
                            hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync((void *)md.prior_mean, E.prior_mean.data(), sizeof(float) * E.dx,
                            hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync((void *)md.prior_sd, E.prior_sd.data(), sizeof(float) * E.dx,
                            hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemsetAsync(D.fstat, 0, sizeof(double) * (size_t)E.d.M * pfk::FREC, s));
    INIT_TRY(hipMemsetAsync(D.emean, 0, sizeof(double) * 2 * (size_t)E.dx, s));
    // every ancestor index is valid from the start
    INIT_TRY(hipMemsetAsync(D.A, 0, sizeof(int32_t) * (size_t)E.d.M * E.d.N, s));
    if (E.lwc) INIT_TRY(pfk::launch_fill_f32(E.lwc, 0.f, (size_t)E.d.M * E.d.N, s));
    // tile maximum keys start empty (key 0; the bits of 0.0f)
    INIT_TRY(pfk::launch_fill_f32((float *)D.mxkey, 0.f, (size_t)E.d.M * E.T, s));
    if (E.grid)
      INIT_TRY(pfk::launch_grid_init(D, D.X[0], s));
    else
      INIT_TRY(pfk::launch_vec_init(D, D.X[0], s));
    if (E.learned) {
      // u = 0 until pf_proposal_set: the bootstrap proposal
      INIT_TRY(hipMemsetAsync(E.params, 0,
                              sizeof(float) * pfk::mlp_nparams(LEARNED_IN, LEARNED_OUT), s));
      INIT_TRY(hipMemcpyAsync(E.nearest, near_host.data(), sizeof(int32_t) * near_host.size(),
                              hipMemcpyHostToDevice, s));
      INIT_TRY(pfk::set_learned_lds_limit());
      // the host vector must outlive the copy
      INIT_TRY(hipStreamSynchronize(s));
    }
  }
  // context arrays: the fused ensemble table, the plan tables, the counter
  {
    pf_status st = PF_OK;
    const CtxSizes z = ctx_sizes(h_models, h_ens, n_ens);
    ctx->d_fens = (pfk::FusedEns *)(ws + base);
    size_t o = base + align_up(sizeof(pfk::FusedEns) * (size_t)n_ens);
    ctx->d_counts = (int32_t **)(ws + o);
    o += align_up(sizeof(int32_t *) * (size_t)n_ens);
    ctx->counts_host.resize((size_t)n_ens);
    for (int e = 0; e < n_ens; ++e) ctx->counts_host[(size_t)e] = ctx->ens[(size_t)e].cnt;
    INIT_TRY(hipMemcpyAsync(ctx->d_counts, ctx->counts_host.data(), sizeof(int32_t *) * (size_t)n_ens,
                            hipMemcpyHostToDevice, s));
    ctx->fz_host.resize((size_t)n_ens);
    for (int e = 0; e < n_ens; ++e) ctx->fz_host[(size_t)e] = ctx->ens[(size_t)e].fz;
    INIT_TRY(hipMemcpyAsync(ctx->d_fens, ctx->fz_host.data(), sizeof(pfk::FusedEns) * (size_t)n_ens,
                            hipMemcpyHostToDevice, s));
    ctx->max_jobs = z.jobs;
    ctx->d_job_base = (pfk::WgJob *)(ws + o);
    o += MAX_CLASSES * align_up(sizeof(pfk::WgJob) * z.jobs);
    for (int w = 0; w < 2; ++w) {
      ctx->d_tiles[w] = (int4 *)(ws + o);
      o += align_up(sizeof(int4) * z.tiles);
    }
    ctx->d_gptab = (int4 *)(ws + o);
    o += align_up(sizeof(int4) * z.gparticles);
    ctx->d_gpart = (int4 *)(ws + o);
    o += align_up(sizeof(int4) * z.gpart_jobs);
    ctx->d_gfold = (int4 *)(ws + o);
    o += align_up(sizeof(int4) * z.gfold_jobs);
    ctx->d_ggens = (int *)(ws + o);
    o += align_up(sizeof(int) * (size_t)n_ens);
    ctx->d_t = (int *)(ws + o);
    o += align_up(sizeof(int));
    INIT_TRY(pfk::set_filter_wg_lds_limit());
    if (st == PF_OK) st = build_plan(ctx, ctx->tuning, s);
    if (st != PF_OK) {
      delete ctx;
      return st;
    }
  }
  // the host copies above must stay valid until the uploads ran
  {
    pf_status st = dev(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != PF_OK) {
      delete ctx;
      return st;
    }
  }
  ctx->t = 1;
  ctx->cur = 0;
  ctx->xbar = 1;
  ctx->pending = false;
  ctx->last_stream = s;
  *out_ctx = ctx;
  return PF_OK;
}

pf_status pf_step(pf_ctx *ctx, const float *d_y, void *stream) {
  if (!ctx) return fail(PF_ERR_STATE, "pf_step before pf_init");
  hipStream_t s = (hipStream_t)stream;
  if (!d_y) {
    if (!ctx->y_all) return fail(PF_ERR_INVALID_ARG, "d_y is NULL and no observations are staged");
    if (ctx->t > ctx->y_T)
      return fail(PF_ERR_INVALID_ARG, "interval %d beyond the %d staged observations", ctx->t,
                  ctx->y_T);
    if ((ctx->options & PF_OPT_GRAPH) && ctx->pending) {
      PF_TRY(graph_step(ctx, s));
      ctx->t += 1;
      return PF_OK;
    }
    d_y = ctx->y_all + (size_t)(ctx->t - 1) * ctx->dy_total;
  }
  if (ctx->options & PF_OPT_FUSED)
    PF_TRY(fused_run(ctx, d_y, s, false));
  else
    PF_TRY(stage_run(ctx, PF_STAGE_ALL, d_y, s));
  ctx->t += 1;
  ctx->d_t_valid = false;
  return PF_OK;
}

pf_status pf_run_stages(pf_ctx *ctx, uint32_t stages, const float *d_y, void *stream) {
  if (!ctx) return fail(PF_ERR_STATE, "pf_run_stages before pf_init");
  if (stages & ~PF_STAGE_ALL) return fail(PF_ERR_INVALID_ARG, "unknown stage bits");
  if ((ctx->options & PF_OPT_FUSED) && (stages & PF_STAGE_RESAMPLE) &&
      !(stages & (PF_STAGE_PROPAGATE | PF_STAGE_WEIGHT))) {
    // resampling (+ gather and estimates) through the fused kernel's phases
    PF_TRY(fused_run(ctx, nullptr, (hipStream_t)stream, true));
    if (stages & PF_STAGE_GATHER) PF_TRY(materialise(ctx, (hipStream_t)stream));
    return PF_OK;
  }
  return stage_run(ctx, stages, d_y, (hipStream_t)stream);
}

pf_status pf_estimate(pf_ctx *ctx, double *d_mean, double *d_mean_w, double *d_logZ,
                      double *d_filter_mean, void *stream) {
  if (!ctx) return fail(PF_ERR_STATE, "pf_estimate before pf_init");
  hipStream_t s = (hipStream_t)stream;
  size_t xo = 0, mo = 0, fo = 0;
  for (Ens &E : ctx->ens) {
    const pfk::EnsDev &D = E.dev;
    if (d_mean)
      PF_HIP(hipMemcpyAsync(d_mean + xo, D.emean, sizeof(double) * E.dx, hipMemcpyDeviceToDevice, s));
    if (d_mean_w)
      PF_HIP(hipMemcpyAsync(d_mean_w + xo, D.emean + E.dx, sizeof(double) * E.dx,
                            hipMemcpyDeviceToDevice, s));
    if (d_logZ)
      PF_HIP(hipMemcpy2DAsync(d_logZ + mo, sizeof(double), D.fstat + 5, sizeof(double) * pfk::FREC,
                              sizeof(double), (size_t)E.d.M, hipMemcpyDeviceToDevice, s));
    if (d_filter_mean)
      PF_HIP(hipMemcpyAsync(d_filter_mean + fo, D.fmean, sizeof(double) * (size_t)E.d.M * E.dx,
                            hipMemcpyDeviceToDevice, s));
    xo += (size_t)E.dx;
    mo += (size_t)E.d.M;
    fo += (size_t)E.d.M * E.dx;
  }
  ctx->last_stream = s;
  return PF_OK;
}

pf_status pf_set_particles(pf_ctx *ctx, int32_t ens, const float *d_x, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_x) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  hipStream_t s = (hipStream_t)stream;
  PF_TRY(materialise(ctx, s));
  const size_t bytes = sizeof(float) * (size_t)E->d.M * E->d.N * E->dx;
  PF_HIP(hipMemcpyAsync(E->dev.X[ctx->cur], d_x, bytes, hipMemcpyDeviceToDevice, s));
  return PF_OK;
}

pf_status pf_get_particles(pf_ctx *ctx, int32_t ens, float *d_x, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_x) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  hipStream_t s = (hipStream_t)stream;
  if (ctx->pending) {
    if (E->grid)
      PF_HIP(pfk::launch_grid_gather(E->dev, E->dev.X[ctx->cur], d_x, s));
    else
      PF_HIP(pfk::launch_vec_gather(E->dev, E->dev.X[ctx->cur], d_x, s));
  } else {
    const size_t bytes = sizeof(float) * (size_t)E->d.M * E->d.N * E->dx;
    PF_HIP(hipMemcpyAsync(d_x, E->dev.X[ctx->cur], bytes, hipMemcpyDeviceToDevice, s));
  }
  return PF_OK;
}

pf_status pf_get_predicted(pf_ctx *ctx, int32_t ens, float *d_x, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_x) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  const size_t bytes = sizeof(float) * (size_t)E->d.M * E->d.N * E->dx;
  PF_HIP(hipMemcpyAsync(d_x, E->dev.X[ctx->xbar], bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_set_predicted(pf_ctx *ctx, int32_t ens, const float *d_x, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_x) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  hipStream_t s = (hipStream_t)stream;
  PF_TRY(materialise(ctx, s));
  ctx->xbar = 1 - ctx->cur;
  const size_t bytes = sizeof(float) * (size_t)E->d.M * E->d.N * E->dx;
  PF_HIP(hipMemcpyAsync(E->dev.X[ctx->xbar], d_x, bytes, hipMemcpyDeviceToDevice, s));
  return PF_OK;
}

pf_status pf_get_logweights(pf_ctx *ctx, int32_t ens, float *d_lw, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_lw) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  PF_HIP(hipMemcpyAsync(d_lw, E->dev.lw, sizeof(float) * (size_t)E->d.M * E->d.N,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_set_logweights(pf_ctx *ctx, int32_t ens, const float *d_lw, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_lw) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  PF_HIP(hipMemcpyAsync(E->dev.lw, d_lw, sizeof(float) * (size_t)E->d.M * E->d.N,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_get_carried_logweights(pf_ctx *ctx, int32_t ens, float *d_lwc, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_lwc) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  if (!E->lwc) return fail(PF_ERR_STATE, "ensemble %d has no ESS threshold", ens);
  PF_HIP(hipMemcpyAsync(d_lwc, E->lwc, sizeof(float) * (size_t)E->d.M * E->d.N,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_set_carried_logweights(pf_ctx *ctx, int32_t ens, const float *d_lwc, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_lwc) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  if (!E->lwc) return fail(PF_ERR_STATE, "ensemble %d has no ESS threshold", ens);
  PF_HIP(hipMemcpyAsync(E->lwc, d_lwc, sizeof(float) * (size_t)E->d.M * E->d.N,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_get_ancestors(pf_ctx *ctx, int32_t ens, int32_t *d_a, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_a) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  PF_HIP(hipMemcpyAsync(d_a, E->dev.A, sizeof(int32_t) * (size_t)E->d.M * E->d.N,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_get_filter_stats(pf_ctx *ctx, int32_t ens, double *d_stats, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_stats) return fail(PF_ERR_INVALID_ARG, "bad context, ensemble or pointer");
  PF_HIP(hipMemcpy2DAsync(d_stats, 4 * sizeof(double), E->dev.fstat, sizeof(double) * pfk::FREC,
                          4 * sizeof(double), (size_t)E->d.M, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_set_interval(pf_ctx *ctx, int32_t t) {
  if (!ctx) return fail(PF_ERR_STATE, "no context");
  if (t < 1) return fail(PF_ERR_INVALID_ARG, "interval index starts at 1");
  ctx->t = t;
  ctx->d_t_valid = false;
  return PF_OK;
}

pf_status pf_set_observations(pf_ctx *ctx, const float *d_y_all, int32_t T) {
  if (!ctx) return fail(PF_ERR_STATE, "no context");
  if (!d_y_all || T < 1) return fail(PF_ERR_INVALID_ARG, "bad observation record");
  int dy = 0;
  for (const Ens &E : ctx->ens) dy += E.dy;
  if (ctx->y_all != d_y_all || ctx->dy_total != dy) drop_graphs(ctx);  // they hold the old pointer
  ctx->y_all = d_y_all;
  ctx->y_T = T;
  ctx->dy_total = dy;
  return PF_OK;
}

pf_status pf_get_interval(const pf_ctx *ctx, int32_t *out_t) {
  if (!ctx || !out_t) return fail(PF_ERR_INVALID_ARG, "NULL argument");
  *out_t = ctx->t;
  return PF_OK;
}

pf_status pf_simulate(pf_ctx *ctx, int32_t ens, uint64_t seed, int32_t T, float *d_x_true,
                      float *d_y, void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E || !d_x_true || !d_y || T < 1) return fail(PF_ERR_INVALID_ARG, "bad simulate arguments");
  if (E->paper)
    PF_HIP(pfk::launch_fhnp_simulate(E->dev, seed, T, d_x_true, d_y, (hipStream_t)stream));
  else if (E->grid)
    PF_HIP(pfk::launch_grid_simulate(E->dev, seed, T, d_x_true, d_y, (hipStream_t)stream));
  else
    PF_HIP(pfk::launch_vec_simulate(E->dev, seed, T, d_x_true, d_y, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                           uint32_t *d_bits, float *d_z, void *stream) {
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(PF_ERR_INVALID_ARG, "n out of range");
  PF_HIP(pfk::launch_philox_stream(seed, c1, c2, c3, n, d_bits, d_z, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_get_tuning(const pf_ctx *ctx, pf_tuning *out) {
  if (!ctx || !out) return fail(PF_ERR_INVALID_ARG, "NULL argument");
  *out = ctx->tuning;
  return PF_OK;
}

pf_status pf_set_tuning(pf_ctx *ctx, const pf_tuning *u, void *stream) {
  if (!ctx || !u) return fail(PF_ERR_INVALID_ARG, "NULL argument");
  PF_TRY(check_tuning(*u));
  hipStream_t s = (hipStream_t)stream;
  // the tables are rewritten in place: let queued work that reads them finish
  if (ctx->last_stream) PF_HIP(hipStreamSynchronize(ctx->last_stream));
  PF_HIP(hipStreamSynchronize(s));
  PF_TRY(build_plan(ctx, *u, s));
  ctx->last_stream = s;
  return PF_OK;
}

pf_status pf_autotune(pf_ctx *ctx, const float *d_y, int32_t reps, void *stream, pf_tuning *out) {
  if (!ctx) return fail(PF_ERR_STATE, "no context");
  if (!(ctx->options & PF_OPT_FUSED)) return fail(PF_ERR_STATE, "the tuning applies to the fused path");
  if (!d_y) return fail(PF_ERR_INVALID_ARG, "the timed intervals need observations");
  if (reps < 1 || reps > 1000) return fail(PF_ERR_INVALID_ARG, "reps out of range");
  hipStream_t s = (hipStream_t)stream;
  if (ctx->last_stream) PF_HIP(hipStreamSynchronize(ctx->last_stream));
  bool any_vec = false, any_small = false, any_grid = !ctx->ggroups.empty(), any_resample = false;
  for (const Ens &E : ctx->ens) {
    if (!E.grid && E.d.N <= pfk::WG_MAX_N) any_vec = true;
    if (E.d.N <= 512) any_small = true;
    if (E.d.N <= pfk::WG_MAX_N) any_resample = true;
  }
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  // wall time of `reps` fused intervals under tuning u (after one warm-up)
  auto measure = [&](const pf_tuning &u, float *ms) -> pf_status {
    PF_HIP(hipStreamSynchronize(s));
    PF_TRY(build_plan(ctx, u, s));
    PF_TRY(fused_run(ctx, d_y, s, false));
    PF_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) PF_TRY(fused_run(ctx, d_y, s, false));
    PF_HIP(hipEventRecord(e1, s));
    PF_HIP(hipEventSynchronize(e1));
    PF_HIP(hipEventElapsedTime(ms, e0, e1));
    return PF_OK;
  };
  pf_tuning best = ctx->tuning;
  float best_ms = 0.f;
  pf_status st = measure(best, &best_ms);
  // coordinate search, one knob at a time in the order of their effect
  auto try_knob = [&](int32_t pf_tuning::*field, std::initializer_list<int> values) {
    for (int v : values) {
      if (st != PF_OK) return;
      if (best.*field == v) continue;
      pf_tuning u = best;
      u.*field = v;
      float ms = 0.f;
      st = measure(u, &ms);
      if (st == PF_OK && ms < best_ms) {
        best_ms = ms;
        best = u;
      }
    }
  };
  if (any_vec) try_knob(&pf_tuning::vec_single_kernel, {0, 1});
  if (any_vec && !best.vec_single_kernel) try_knob(&pf_tuning::prop_tile, {64, 128, 256});
  if (any_resample) {
    if (any_small) try_knob(&pf_tuning::resample_bd_min, {64, 128, 256, 512});
    try_knob(&pf_tuning::resample_bd_min, {1024});
  }
  if (any_grid) try_knob(&pf_tuning::grid_blocks_per_cu, {0, 1, 2, 4, 8});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  PF_TRY(st);
  PF_HIP(hipStreamSynchronize(s));
  PF_TRY(build_plan(ctx, best, s));
  // the timed intervals moved the filters: back to the prior draw at t = 1
  PF_TRY(reset_filters(ctx, s));
  if (out) *out = best;
  ctx->last_stream = s;
  return PF_OK;
}

int32_t pf_mlp_nparams(int32_t in_dim, int32_t out_dim) {
  if (in_dim < 1 || in_dim > 31 || out_dim < 1 || out_dim > 4) return -1;
  return pfk::mlp_nparams(in_dim, out_dim);
}

pf_status pf_proposal_set(pf_ctx *ctx, int32_t ens, const float *d_params, int64_t n_params,
                          void *stream) {
  Ens *E = get_ens(ctx, ens);
  if (!E) return fail(PF_ERR_INVALID_ARG, "bad ensemble index");
  if (!E->learned) return fail(PF_ERR_STATE, "ensemble %d was not created with PF_ENS_LEARNED", ens);
  if (!d_params || n_params != pfk::mlp_nparams(LEARNED_IN, LEARNED_OUT))
    return fail(PF_ERR_INVALID_ARG, "expected %d parameters",
                pfk::mlp_nparams(LEARNED_IN, LEARNED_OUT));
  PF_HIP(hipMemcpyAsync(E->params, d_params, sizeof(float) * (size_t)n_params,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_mlp_forward(const float *d_params, int32_t in_dim, int32_t out_dim, const float *d_x,
                         int64_t rows, float *d_out, void *stream) {
  if (pf_mlp_nparams(in_dim, out_dim) < 0)
    return fail(PF_ERR_INVALID_ARG, "in_dim must be in [1, 31] and out_dim in [1, 4]");
  if (rows < 0) return fail(PF_ERR_INVALID_ARG, "rows < 0");
  if (rows > 0 && (!d_params || !d_x || !d_out)) return fail(PF_ERR_INVALID_ARG, "NULL buffer");
  PF_HIP(pfk::launch_mlp_forward(d_params, in_dim, out_dim, d_x, rows, d_out, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_mlp_grad_work_bytes(int32_t in_dim, int32_t out_dim, int64_t rows, size_t *out_bytes) {
  if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
  const int np = pf_mlp_nparams(in_dim, out_dim);
  if (np < 0) return fail(PF_ERR_INVALID_ARG, "in_dim must be in [1, 31] and out_dim in [1, 4]");
  if (rows < 1) return fail(PF_ERR_INVALID_ARG, "rows < 1");
  *out_bytes = sizeof(float) * pfk::mlp_grad_work_floats((rows + 15) / 16, np);
  return PF_OK;
}

pf_status pf_mlp_loss_grad(const float *d_params, int32_t in_dim, int32_t out_dim, const float *d_x,
                           const float *d_target, int64_t rows, float *d_grad, float *d_loss,
                           void *d_work, size_t work_bytes, void *stream) {
  size_t need = 0;
  PF_TRY(pf_mlp_grad_work_bytes(in_dim, out_dim, rows, &need));
  if (!d_params || !d_x || !d_target || !d_grad) return fail(PF_ERR_INVALID_ARG, "NULL buffer");
  if (!d_work || work_bytes < need)
    return fail(PF_ERR_WORKSPACE, "work buffer too small: %zu < %zu bytes", work_bytes, need);
  PF_HIP(pfk::launch_mlp_grad_rows(d_params, in_dim, out_dim, d_x, d_target, rows, (float *)d_work,
                                   d_grad, d_loss, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_mlp_loss_grad_noalloc(const float *d_params, int32_t in_dim, int32_t out_dim,
                                   const float *d_x, const float *d_target, int64_t rows,
                                   float *d_grad, float *d_loss, void *stream) {
  size_t need = 0;
  PF_TRY(pf_mlp_grad_work_bytes(in_dim, out_dim, rows, &need));
  if (!d_params || !d_x || !d_target || !d_grad) return fail(PF_ERR_INVALID_ARG, "NULL buffer");
  if (need > PF_MLP_GRAD_STATIC_BYTES)
    return fail(PF_ERR_WORKSPACE,
                "%lld rows need %zu bytes of partial gradients; the static buffer holds %zu "
                "(use pf_mlp_loss_grad with a work buffer)",
                (long long)rows, need, (size_t)PF_MLP_GRAD_STATIC_BYTES);
  float *scratch = nullptr;
  PF_HIP(pfk::mlp_grad_scratch(&scratch));
  PF_HIP(pfk::launch_mlp_grad_rows(d_params, in_dim, out_dim, d_x, d_target, rows, scratch, d_grad,
                                   d_loss, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t n,
                       double lr, double beta1, double beta2, double eps, int32_t t, void *stream) {
  if (n < 1 || n > (1 << 30)) return fail(PF_ERR_INVALID_ARG, "n out of range");
  if (!d_params || !d_grad || !d_m || !d_v) return fail(PF_ERR_INVALID_ARG, "NULL buffer");
  if (t < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(PF_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  PF_HIP(pfk::launch_adam(d_params, d_grad, d_m, d_v, (int)n, lr, beta1, beta2, eps, t,
                          (hipStream_t)stream));
  return PF_OK;
}

}  // extern "C"

namespace {

// Layout of the training workspace of an FH-N model.
struct TrainLayout {
  size_t obs, pmean, psd, nearest, starts, traj, ys, partial, mo, ve, end;
  int nn, n_traj, np;
};

pf_status train_check(const pf_model_desc *m, const pf_train_desc *d) {
  if (!m || !d) return fail(PF_ERR_INVALID_ARG, "NULL descriptor");
  PF_TRY(check_model(*m, 0));
  if (m->kind != PF_MODEL_FHN || m->grid_j > LEARNED_MAX_J || (m->grid_j % 4) != 0)
    return fail(PF_ERR_UNSUPPORTED, "training needs an FH-N model with J a multiple of 4, <= %d",
                LEARNED_MAX_J);
  if (d->n_runs < 1 || d->run_len < 1 || (int64_t)d->n_runs * d->run_len > (1 << 24))
    return fail(PF_ERR_INVALID_ARG, "bad n_runs / run_len");
  if (d->batch_tiles < 1 || d->batch_tiles > (1 << 20))
    return fail(PF_ERR_INVALID_ARG, "batch_tiles out of range");
  if (!(d->lr > 0.0) || !(d->beta1 >= 0.0 && d->beta1 < 1.0) ||
      !(d->beta2 >= 0.0 && d->beta2 < 1.0) || !(d->eps > 0.0))
    return fail(PF_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  return PF_OK;
}

TrainLayout train_layout(const pf_model_desc &m, const pf_train_desc &d) {
  TrainLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.nn = m.grid_j * m.grid_j;
  L.n_traj = d.n_runs * d.run_len;
  L.np = pfk::mlp_nparams(LEARNED_IN, LEARNED_OUT);
  const size_t dx = (size_t)m.state_dim;
  L.obs = take(sizeof(int32_t) * (size_t)m.obs_dim);
  L.pmean = take(sizeof(float) * dx);
  L.psd = take(sizeof(float) * dx);
  L.nearest = take(sizeof(int32_t) * (size_t)L.nn);
  L.starts = take(sizeof(float) * (size_t)L.n_traj * dx);
  L.traj = take(sizeof(float) * (size_t)L.n_traj * m.steps_per_obs * dx);
  L.ys = take(sizeof(float) * (size_t)L.n_traj * m.obs_dim);
  L.partial = take(sizeof(float) * pfk::mlp_grad_work_floats(d.batch_tiles, L.np));
  L.mo = take(sizeof(float) * (size_t)L.np);
  L.ve = take(sizeof(float) * (size_t)L.np);
  L.end = o;
  return L;
}

pfk::ModelDev train_model_dev(const pf_model_desc &m, const TrainLayout &L, char *ws) {
  pfk::ModelDev md{};
  md.kind = m.kind;
  md.dx = m.state_dim;
  md.J = m.grid_j;
  md.S = m.steps_per_obs;
  md.dy = m.obs_dim;
  md.h = (float)m.h;
  md.p0 = (float)m.params[0];
  md.p1 = (float)m.params[1];
  md.p2 = (float)m.params[2];
  md.p3 = (float)m.params[3];
  md.sq0 = (float)(m.noise_sd[0] * std::sqrt(m.h));
  md.sq1 = (float)(m.noise_sd[1] * std::sqrt(m.h));
  md.inv2var = (float)(1.0 / (2.0 * m.obs_var));
  md.obs_sd = (float)std::sqrt(m.obs_var);
  md.obs_idx = (const int32_t *)(ws + L.obs);
  md.prior_mean = (const float *)(ws + L.pmean);
  md.prior_sd = (const float *)(ws + L.psd);
  return md;
}

}  // namespace

extern "C" {

pf_status pf_train_workspace_bytes(const pf_model_desc *h_model, const pf_train_desc *d,
                                   size_t *out_bytes) {
  if (!out_bytes) return fail(PF_ERR_INVALID_ARG, "out_bytes is NULL");
  PF_TRY(train_check(h_model, d));
  *out_bytes = train_layout(*h_model, *d).end;
  return PF_OK;
}

pf_status pf_train_buffers(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                           float **d_starts, float **d_traj, float **d_y) {
  PF_TRY(train_check(h_model, d));
  if (!d_work) return fail(PF_ERR_INVALID_ARG, "NULL workspace");
  const TrainLayout L = train_layout(*h_model, *d);
  char *ws = (char *)d_work;
  if (d_starts) *d_starts = (float *)(ws + L.starts);
  if (d_traj) *d_traj = (float *)(ws + L.traj);
  if (d_y) *d_y = (float *)(ws + L.ys);
  return PF_OK;
}

pf_status pf_train_data(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                        size_t work_bytes, void *stream) {
  PF_TRY(train_check(h_model, d));
  const TrainLayout L = train_layout(*h_model, *d);
  if (!d_work || ((uintptr_t)d_work % ALIGN) != 0 || work_bytes < L.end)
    return fail(PF_ERR_WORKSPACE, "training workspace must be 256-byte aligned and %zu bytes", L.end);
  const pf_model_desc &m = *h_model;
  char *ws = (char *)d_work;
  hipStream_t s = (hipStream_t)stream;
  const pfk::ModelDev md = train_model_dev(m, L, ws);
  std::vector<float> pm((size_t)m.state_dim), psd((size_t)m.state_dim);
  for (int k = 0; k < m.state_dim; ++k) {
    pm[(size_t)k] = (float)m.h_prior_mean[k];
    psd[(size_t)k] = (float)m.h_prior_sd[k];
  }
  const int J = m.grid_j;
  std::vector<int32_t> near((size_t)L.nn);
  for (int n = 0; n < L.nn; ++n) {
    const int i = n / J, j = n % J;
    long best = -1;
    for (int o = 0; o < m.obs_dim; ++o) {
      const int r = m.h_obs_index[o] / J, c = m.h_obs_index[o] % J;
      const long d2 = (long)(i - r) * (i - r) + (long)(j - c) * (j - c);
      if (best < 0 || d2 < best) {
        best = d2;
        near[(size_t)n] = o;
      }
    }
  }
  PF_HIP(hipMemcpyAsync(ws + L.obs, m.h_obs_index, sizeof(int32_t) * m.obs_dim,
                        hipMemcpyHostToDevice, s));
  PF_HIP(hipMemcpyAsync(ws + L.pmean, pm.data(), sizeof(float) * pm.size(), hipMemcpyHostToDevice, s));
  PF_HIP(hipMemcpyAsync(ws + L.psd, psd.data(), sizeof(float) * psd.size(), hipMemcpyHostToDevice, s));
  PF_HIP(hipMemcpyAsync(ws + L.nearest, near.data(), sizeof(int32_t) * near.size(),
                        hipMemcpyHostToDevice, s));
  const pfk::Key key = pfk::make_key(d->seed);
  PF_HIP(pfk::launch_train_sim(md, key, 0, d->n_runs, d->run_len, nullptr,
                               (float *)(ws + L.starts), nullptr, s));
  PF_HIP(pfk::launch_train_sim(md, key, 1, L.n_traj, 1, (const float *)(ws + L.starts),
                               (float *)(ws + L.traj), (float *)(ws + L.ys), s));
  // the host staging vectors must outlive the copies
  PF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

pf_status pf_train_steps(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                         size_t work_bytes, float *d_params, int32_t first_step, int32_t n_steps,
                         float *d_loss, void *stream) {
  PF_TRY(train_check(h_model, d));
  const TrainLayout L = train_layout(*h_model, *d);
  if (!d_work || ((uintptr_t)d_work % ALIGN) != 0 || work_bytes < L.end)
    return fail(PF_ERR_WORKSPACE, "training workspace must be 256-byte aligned and %zu bytes", L.end);
  if (!d_params) return fail(PF_ERR_INVALID_ARG, "NULL parameters");
  if (first_step < 1 || n_steps < 0) return fail(PF_ERR_INVALID_ARG, "bad step range");
  const pf_model_desc &m = *h_model;
  char *ws = (char *)d_work;
  hipStream_t s = (hipStream_t)stream;
  const pfk::ModelDev md = train_model_dev(m, L, ws);
  const pfk::Key key = pfk::make_key(d->seed);
  float *mo = (float *)(ws + L.mo), *ve = (float *)(ws + L.ve);
  if (first_step == 1) {
    PF_HIP(hipMemsetAsync(mo, 0, sizeof(float) * (size_t)L.np, s));
    PF_HIP(hipMemsetAsync(ve, 0, sizeof(float) * (size_t)L.np, s));
  }
  const float tsv = (float)(m.noise_sd[0] / std::sqrt(m.h));
  const float tsw = (float)(m.noise_sd[1] / std::sqrt(m.h));
  for (int k = 0; k < n_steps; ++k)
    PF_HIP(pfk::launch_train_fhn_step(
        md, key, (const float *)(ws + L.traj), (const float *)(ws + L.ys),
        (const int32_t *)(ws + L.nearest), L.n_traj, first_step + k, d->batch_tiles, tsv, tsw,
        d_params, (float *)(ws + L.partial), mo, ve, d->lr, d->beta1, d->beta2, d->eps,
        d_loss ? d_loss + k : nullptr, nullptr, 1, s));
  return PF_OK;
}

pf_status pf_train_grad(const pf_model_desc *h_model, const pf_train_desc *d, void *d_work,
                        size_t work_bytes, const float *d_params, int32_t step, float *d_grad,
                        float *d_loss, void *stream) {
  PF_TRY(train_check(h_model, d));
  const TrainLayout L = train_layout(*h_model, *d);
  if (!d_work || ((uintptr_t)d_work % ALIGN) != 0 || work_bytes < L.end)
    return fail(PF_ERR_WORKSPACE, "training workspace must be 256-byte aligned and %zu bytes", L.end);
  if (!d_params || !d_grad) return fail(PF_ERR_INVALID_ARG, "NULL buffer");
  if (step < 1) return fail(PF_ERR_INVALID_ARG, "step < 1");
  const pf_model_desc &m = *h_model;
  char *ws = (char *)d_work;
  const pfk::ModelDev md = train_model_dev(m, L, ws);
  PF_HIP(pfk::launch_train_fhn_step(
      md, pfk::make_key(d->seed), (const float *)(ws + L.traj), (const float *)(ws + L.ys),
      (const int32_t *)(ws + L.nearest), L.n_traj, step, d->batch_tiles,
      (float)(m.noise_sd[0] / std::sqrt(m.h)), (float)(m.noise_sd[1] / std::sqrt(m.h)),
      const_cast<float *>(d_params), (float *)(ws + L.partial), nullptr, nullptr, 0.0, 0.0, 0.0,
      0.0, d_loss, d_grad, 0, (hipStream_t)stream));
  return PF_OK;
}

pf_status pf_set_profiling(pf_ctx *ctx, int32_t enable) {
  if (!ctx) return fail(PF_ERR_STATE, "no context");
  ctx->profiling = enable != 0;
  return PF_OK;
}

pf_status pf_read_profile(pf_ctx *ctx, double *out_ms, int64_t *out_launches) {
  if (!ctx || !out_ms || !out_launches) return fail(PF_ERR_INVALID_ARG, "NULL argument");
  double total = 0.0;
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    PF_HIP(hipEventSynchronize(ctx->ev_stop[i]));
    float ms = 0.f;
    PF_HIP(hipEventElapsedTime(&ms, ctx->ev_start[i], ctx->ev_stop[i]));
    total += (double)ms;
  }
  *out_ms = total;
  *out_launches = (int64_t)ctx->ev_used;
  ctx->ev_used = 0;
  return PF_OK;
}

pf_status pf_sync(pf_ctx *ctx) {
  if (!ctx) return fail(PF_ERR_STATE, "no context");
  PF_HIP(hipStreamSynchronize(ctx->last_stream));
  PF_HIP(hipGetLastError());
  return PF_OK;
}

void pf_destroy(pf_ctx *ctx) {
  if (!ctx) return;
  // wait for everything the context queued before its streams, events and
  // graphs go: the caller's last stream (which a replayed graph and the
  // joined side stream end on) and the context's own streams
  if (ctx->last_stream) (void)hipStreamSynchronize(ctx->last_stream);
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);
  if (ctx->cap_stream) (void)hipStreamSynchronize(ctx->cap_stream);
  delete ctx;
}

const char *pf_status_str(pf_status s) {
  switch (s) {
    case PF_OK: return "ok";
    case PF_ERR_INVALID_ARG: return "invalid argument";
    case PF_ERR_UNSUPPORTED: return "unsupported";
    case PF_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PF_ERR_DEVICE: return "device error";
    case PF_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

const char *pf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
