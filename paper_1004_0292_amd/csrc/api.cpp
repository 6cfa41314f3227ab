// Host runtime and C-ABI of the sscg library (declared in include/sscg.h).
//
// A context owns one lattice: its packed gauge field (FP64 18-real and, for the
// mixed mode, FP32 18- or 12-real), and the solver workspaces, grown on demand
// and reused. The shifted CG (Sec. 2.2) runs as a loop of grouped launches
// (dslash, seed step length and residual, fused shift update with the shift
// scalars) whose scalar state lives in device memory; the host only polls the
// per-source "done" words every poll_every iterations, and the iterations in
// between replay as one HIP graph. Several contexts can be solved together (sscg_batch_solve): each
// stage is then one launch whose blocks are split over the problems.
#include "sscg.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host_math.h"
#include "sscg_internal.h"

using namespace sscg;
using cd = std::complex<double>;

static std::string g_global_err;
static constexpr int kEptHost = 2;  // entries per thread of the streaming kernels (vec.hip)

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct Tune {
  int nr = 2;       // sources per dslash thread
  int bs = 256;     // sites per dslash block
  int wbatch = 8;   // shifts per block of the fused shift update
  int xcd = 1;      // XCD-aware block order in the dslash
  int unroll = 2;   // shifts whose loads a shift-update thread issues together
  int nt = 0;       // non-temporal access to the shift vectors
  int ct = 0;       // t-slices per block of the tile dslash (0: site-parallel kernel)
  int tbs = 0;      // sites (threads) per tile of the tile dslash
  int border = 0;   // shift-update block order (1: the shift batches of an entry chunk adjacent)
};

enum Stage { ST_DSLASH = 0, ST_ALPHA, ST_RUPD, ST_SCAL, ST_SHIFT, ST_RU, ST_LOOP, ST_PASS, ST_N = 8 };

struct sscg_ctx {
  int device = 0;
  hipStream_t user = nullptr;   // stream given by the caller
  hipStream_t work = nullptr;   // private stream (graph capture needs a non-null stream)
  hipEvent_t ev_sync = nullptr;
  int dims[4] = {0, 0, 0, 0};
  int V = 0;
  int64_t n = 0;
  double kappa = 0.0;
  DevBuf g64, g32;
  int link_reals = 18;
  bool have_gauge = false;
  std::string err;
  // launch shapes: defaults, overridden by SSCG_NR / SSCG_BS / SSCG_WBATCH / SSCG_XCD,
  // or chosen per problem shape by the autotuner (SSCG_AUTOTUNE=0 disables it)
  Tune tune;
  bool autotune = true;
  int dorder = 1;    // dslash block order (1: all source groups of a site tile adjacent)
  int max_lds = 65536;  // dynamic LDS limit per block (bytes)
  std::map<std::string, Tune> tuned;
  // solver workspaces
  DevBuf v64, r64, p64, q64, W, r32, p32, q32, rbase, xpart64, xpart32, tmp, pq_part, rr_part, seed,
      shift, zdev, small, cmom, Ybuf, Sbuf, Qbuf, AQbuf, Xbuf, AXbuf, Accbuf, apply_in, apply_out, trpart, momtab, ring;
  SeedState *seed_host = nullptr;
  int seed_host_cap = 0;
  // profiling
  int profiling = 0;  // 0 off, 1 every launch, k > 1 every k-th iteration in graphs
  double stage_ms[ST_N] = {};
  int64_t sweep_bytes = 0;  // algorithmic HBM bytes of the block sweeps of the last solve
  int64_t stage_calls[ST_N] = {};
  int64_t stage_launched[ST_N] = {};  // launches of each stage in the last solve
  std::vector<hipEvent_t> events;
  std::vector<double> hstage;  // host staging of small matrices sent to the device
  // solve-loop graphs kept across solves (FP64 and FP32 phase), with the bytes of
  // everything the capture depended on; a solve of the same shape on the same
  // buffers replays them without capturing again
  struct CachedGraph {
    std::string key;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;  // timing marks recorded by the graph (profiling)
    std::vector<int> stages;
    std::vector<int> its;        // iteration (in the chunk) of each timing mark
    bool timed = false;
  } graphs[2];
};

static int fail(sscg_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_global_err = msg;
  return code;
}
#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail(ctx, SSCG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define CHK(call)             \
  do {                        \
    int s_ = (call);          \
    if (s_ != SSCG_OK) return s_; \
  } while (0)

static int ensure(sscg_ctx *c, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return SSCG_OK;
  if (b.p) {
    hipStreamSynchronize(c->work);
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SSCG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return SSCG_OK;
}
static void release(DevBuf &b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

static int env_int(const char *name, int dflt) {
  const char *s = getenv(name);
  return s ? atoi(s) : dflt;
}

extern "C" {

const char *sscg_global_error(void) { return g_global_err.c_str(); }
const char *sscg_last_error(const sscg_ctx *c) { return c ? c->err.c_str() : g_global_err.c_str(); }

int sscg_create(sscg_ctx **out, const int32_t dims[4], double kappa, double r, int32_t device,
                void *hip_stream) {
  if (!out || !dims) return fail(nullptr, SSCG_EINVAL, "null argument");
  *out = nullptr;
  for (int i = 0; i < 4; ++i)
    if (dims[i] <= 0) return fail(nullptr, SSCG_EINVAL, "lattice extents must be positive");
  if (r != 1.0) return fail(nullptr, SSCG_EINVAL, "only the Wilson parameter r = 1 is implemented");
  const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
  if (V > (int64_t)1 << 30) return fail(nullptr, SSCG_EINVAL, "lattice too large");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(nullptr, SSCG_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, SSCG_EINVAL, "bad device index");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, SSCG_EDEVICE, "hipSetDevice failed");
  auto *c = new sscg_ctx();
  c->device = device;
  c->user = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(nullptr, SSCG_EDEVICE, "stream creation failed");
  }
  for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
      c->max_lds = v;
    else
      (void)hipGetLastError();
  }
  c->V = (int)V;
  c->n = 12 * V;
  c->kappa = kappa;
  c->tune.nr = env_int("SSCG_NR", 2);
  c->tune.bs = env_int("SSCG_BS", 256);
  c->tune.wbatch = env_int("SSCG_WBATCH", 8);
  c->tune.xcd = env_int("SSCG_XCD", 1);
  c->tune.unroll = env_int("SSCG_UNROLL", 2);
  c->tune.ct = env_int("SSCG_CT", 0);
  c->tune.tbs = env_int("SSCG_TBS", 256);
  c->tune.border = env_int("SSCG_BORDER", 0) ? 1 : 0;
  c->dorder = env_int("SSCG_DORDER", 1);
  if (c->dorder < 0 || c->dorder > 2) c->dorder = 1;
  if (c->tune.ct < -1) c->tune.ct = 0;
  c->tune.nt = env_int("SSCG_NT", 0);
  c->autotune = env_int("SSCG_AUTOTUNE", 1) != 0 && !getenv("SSCG_NR") && !getenv("SSCG_BS") &&
                !getenv("SSCG_WBATCH") && !getenv("SSCG_XCD") && !getenv("SSCG_UNROLL") && !getenv("SSCG_NT") && !getenv("SSCG_CT") &&
                !getenv("SSCG_TBS") && !getenv("SSCG_BORDER");
  if (c->tune.nr != 1 && c->tune.nr != 2 && c->tune.nr != 4) c->tune.nr = 2;
  if (c->tune.bs != 64 && c->tune.bs != 128 && c->tune.bs != 256) c->tune.bs = 256;
  if (c->tune.wbatch < 1) c->tune.wbatch = 8;
  if (c->tune.wbatch > kMaxWBatch) c->tune.wbatch = kMaxWBatch;  // the update kernel stages a batch in LDS
  *out = c;
  return SSCG_OK;
}

void sscg_destroy(sscg_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->work);
  DevBuf *bufs[] = {&c->g64, &c->g32, &c->v64, &c->r64, &c->p64, &c->q64, &c->W, &c->r32, &c->p32,
                    &c->q32, &c->rbase, &c->xpart64, &c->xpart32, &c->tmp, &c->pq_part, &c->rr_part,
                    &c->seed, &c->shift, &c->zdev, &c->small, &c->cmom, &c->Ybuf, &c->Sbuf, &c->Qbuf, &c->AQbuf,
                    &c->Xbuf, &c->AXbuf, &c->Accbuf, &c->apply_in, &c->apply_out, &c->trpart, &c->momtab, &c->ring};
  for (DevBuf *b : bufs) release(*b);
  if (c->seed_host) hipHostFree(c->seed_host);
  for (hipEvent_t e : c->events) hipEventDestroy(e);
  for (auto &g : c->graphs) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    for (hipEvent_t e : g.ev) hipEventDestroy(e);
  }
  hipEventDestroy(c->ev_sync);
  hipStreamDestroy(c->work);
  delete c;
}

void sscg_default_opts(sscg_solve_opts *o) {
  if (!o) return;
  o->tol = 1e-12;
  o->maxiter = 100000;
  o->prec = SSCG_FP64;
  o->ru_interval = 50;
  o->poll_every = 50;
  o->switch_tol = 1e-6;
  o->use_graph = 1;
  o->pad = 0;
  o->true_factor = 100.0;
}

int sscg_set_gauge(sscg_ctx *c, const double *U, int32_t link_reals) {
  if (!c || !U) return fail(c, SSCG_EINVAL, "null argument");
  if (link_reals != 18 && link_reals != 12) return fail(c, SSCG_EINVAL, "link_reals must be 18 or 12");
  HIPCHK(c, hipSetDevice(c->device));
  const int V = c->V;
  // host conversion canonical [4][V][3][3] -> planar [4][9][V] (FP64) and [4][LR/2][V] (FP32)
  std::vector<double> h64((size_t)4 * 9 * V * 2);
  std::vector<float> h32((size_t)4 * (link_reals / 2) * V * 2);
  for (int mu = 0; mu < 4; ++mu)
    for (int s = 0; s < V; ++s)
      for (int e = 0; e < 9; ++e) {
        const double re = U[2 * (((size_t)mu * V + s) * 9 + e)];
        const double im = U[2 * (((size_t)mu * V + s) * 9 + e) + 1];
        const size_t o = ((size_t)mu * 9 + e) * V + s;
        h64[2 * o] = re;
        h64[2 * o + 1] = im;
        if (e < link_reals / 2) {
          const size_t o32 = ((size_t)mu * (link_reals / 2) + e) * V + s;
          h32[2 * o32] = (float)re;
          h32[2 * o32 + 1] = (float)im;
        }
      }
  CHK(ensure(c, c->g64, h64.size() * sizeof(double)));
  CHK(ensure(c, c->g32, h32.size() * sizeof(float)));
  HIPCHK(c, hipStreamSynchronize(c->work));
  HIPCHK(c, hipMemcpy(c->g64.p, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->g32.p, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice));
  c->link_reals = link_reals;
  c->have_gauge = true;
  return SSCG_OK;
}

int sscg_set_profiling(sscg_ctx *c, int32_t on) {
  if (!c) return SSCG_EINVAL;
  if (on < 0) return fail(c, SSCG_EINVAL, "profiling level must be >= 0");
  c->profiling = on;
  return SSCG_OK;
}
int sscg_stage_times(const sscg_ctx *c, double ms[8], int64_t calls[8]) {
  if (!c || !ms || !calls) return SSCG_EINVAL;
  for (int i = 0; i < ST_N; ++i) {
    ms[i] = c->stage_ms[i];
    calls[i] = c->stage_calls[i];
  }
  return SSCG_OK;
}
int sscg_sweep_bytes(const sscg_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return SSCG_EINVAL;
  *bytes = c->sweep_bytes;
  return SSCG_OK;
}
int sscg_stage_launches(const sscg_ctx *c, int64_t launched[8]) {
  if (!c || !launched) return SSCG_EINVAL;
  for (int i = 0; i < ST_N; ++i) launched[i] = c->stage_launched[i];
  return SSCG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// internal helpers

// Tile of tbs sites for the tile dslash on this lattice: whole x-rows, ty | Ly,
// tz | Lz, Lx ty tz = tbs (a multiple of 64, at most 1024), LDS for nr sources of
// FP64 or FP32 spinors within the device limit; among the shapes, the one with the
// fewest face sites. Returns false if there is none.
static bool tile_shape(const sscg_ctx *c, int tbs, int nr, int prec, int &ty, int &tz) {
  const int Lx = c->dims[0], Ly = c->dims[1], Lz = c->dims[2];
  if (tbs < 64 || tbs > 1024 || tbs % 64 || tbs % Lx) return false;
  const size_t lds = (size_t)nr * 12 * tbs * (prec == 0 ? 16 : 8);
  if (lds > (size_t)c->max_lds) return false;
  const int k = tbs / Lx;
  double best = 1e30;
  for (int a = 1; a <= Ly && a <= k; ++a) {
    if (Ly % a || k % a) continue;
    const int bz = k / a;
    if (bz > Lz || Lz % bz) continue;
    const double f = (a == Ly ? 0.0 : 1.0 / a) + (bz == Lz ? 0.0 : 1.0 / bz);
    if (f < best) {
      best = f;
      ty = a;
      tz = bz;
    }
  }
  return best < 1e29;
}
// site blocks per source group of the dslash: 64-site blocks of the direction-split
// kernel (ct < 0), one thread per site (ct = 0), or tiles times t-ranges of the tile
// kernel (ct > 0)
static int nblk_site(const sscg_ctx *c, int bs, int ct, int ty, int tz) {
  if (ct < 0) return (c->V + 63) / 64;
  if (ct == 0) return (c->V + bs - 1) / bs;
  const int Lt = c->dims[3];
  return (c->dims[1] / ty) * (c->dims[2] / tz) * ((Lt + ct - 1) / ct);
}
static int nblk_vec(const sscg_ctx *c) { return (int)((c->n + kBlock * kEptHost - 1) / (kBlock * kEptHost)); }
constexpr int kMaxRR = 256;  // blocks (and <r, r> partials) per source of the seed passes

// FP64 dslash of nsrc planar vectors: out = A in (mode 0) or sigma in - A in (mode 1)
static void dslash_with(sscg_ctx *c, const Tune &t, const void *in, void *out, int nsrc, int prec, int mode,
                        double sigma, double *partial, const SeedState *seed, hipStream_t st) {
  DslashBatch b{};
  DslashJob &j = b.job[0];
  j.in = in;
  j.out = out;
  j.gauge = prec == 0 ? c->g64.p : c->g32.p;
  j.partial = partial;
  j.seed = const_cast<SeedState *>(seed);  // read only: no shift table, so no commit
  j.kappa = c->kappa;
  j.sigma = sigma;
  for (int i = 0; i < 4; ++i) j.dims[i] = c->dims[i];
  j.V = c->V;
  j.nsrc = nsrc;
  int ct = t.ct, ty = 0, tz = 0;
  if (ct > 0 && !tile_shape(c, t.tbs, t.nr, prec, ty, tz)) ct = 0;
  if (ct < 0 && t.nr > 2) ct = 0;
  j.nblk_site = nblk_site(c, t.bs, ct, ty, tz);
  j.block_begin = 0;
  j.nblocks = j.nblk_site * ((nsrc + t.nr - 1) / t.nr);
  j.mode = mode;
  j.ct = ct;
  j.ty = ty;
  j.tz = tz;
  j.order = c->dorder;
  b.njobs = 1;
  b.total_blocks = j.nblocks;
  launch_dslash(b, prec, t.nr, prec == 0 ? 18 : c->link_reals, t.bs, t.xcd, ct, st);
}

// A launch shape whose launch the runtime rejected (kTuneFailed) never wins a search.
constexpr double kTuneFailed = 1e300;

// Mean duration (ms) of reps launches after one warm-up launch, from HIP events on
// events e0, e1; kTuneFailed if any launch was rejected (the error is cleared).
template <typename F>
static double time_with_events(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F &&launch, int reps) {
  (void)hipGetLastError();
  launch();
  if (hipGetLastError() != hipSuccess) return kTuneFailed;
  hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  const hipError_t le = hipGetLastError();
  hipEventRecord(e1, st);
  hipEventSynchronize(e1);
  if (le != hipSuccess) return kTuneFailed;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
    (void)hipGetLastError();
    return kTuneFailed;
  }
  return ms / reps;
}
template <typename F>
static double time_launches(hipStream_t st, F &&launch, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return kTuneFailed;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return kTuneFailed;
  }
  const double t = time_with_events(st, e0, e1, launch, reps);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return t;
}

// A launch shape replaces the best one found so far only when it is at least 3 %
// faster, so shapes within timing noise of each other do not flip between runs
// (candidates are tried in a fixed order).
constexpr double kTuneMargin = 0.97;

// Second round of a shape search: the kRefine fastest shapes of the first round are
// timed again with more launches, twice, and the shortest of those times decides
// (the first round's short timings only preselect).
constexpr int kRefine = 4;
struct Trial {
  double t;
  int order;
  Tune cd;
};
template <typename F>
static Tune refine_shapes(std::vector<Trial> &trials, const Tune &fallback, F &&time_shape) {
  trials.erase(std::remove_if(trials.begin(), trials.end(), [](const Trial &t) { return t.t >= kTuneFailed; }),
               trials.end());
  if (trials.empty()) return fallback;
  std::sort(trials.begin(), trials.end(),
            [](const Trial &a, const Trial &b) { return a.t < b.t || (a.t == b.t && a.order < b.order); });
  if (trials.size() > (size_t)kRefine) trials.resize(kRefine);
  std::sort(trials.begin(), trials.end(), [](const Trial &a, const Trial &b) { return a.order < b.order; });
  Tune best = trials[0].cd;
  double tbest = 1e300;
  for (const Trial &tr : trials) {
    const double t = std::min(time_shape(tr.cd), time_shape(tr.cd));
    if (t >= kTuneFailed) continue;
    if (t < kTuneMargin * tbest || tbest == 1e300) {
      tbest = t;
      best = tr.cd;
    }
  }
  return best;
}

// Dslash launch shape for out = A in on nsrc vectors outside a solve (apply_A, true
// residuals, Rayleigh-Ritz products): with autotuning on, every shape of the
// site-parallel and tile kernels is timed once on the caller's buffers (out is
// rewritten by the real launch that follows) and the fastest is kept per
// (precision, nsrc).
static Tune apply_tune(sscg_ctx *c, const void *in, void *out, int nsrc, int prec, hipStream_t st) {
  if (!c->autotune) return c->tune;
  const std::string key = "apply|" + std::to_string(prec) + "|" + std::to_string(nsrc);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return it->second;
  Tune cand = c->tune;
  std::vector<Trial> trials;
  auto time_shape = [&](const Tune &cd, int reps) {
    return time_launches(st, [&] { dslash_with(c, cd, in, out, nsrc, prec, 0, 0.0, nullptr, nullptr, st); }, reps);
  };
  auto try_shape = [&](const Tune &cd) {
    int ty, tz;
    if (cd.ct > 0 && !tile_shape(c, cd.tbs, cd.nr, prec, ty, tz)) return;
    trials.push_back({time_shape(cd, 3), (int)trials.size(), cd});
  };
  for (int nr : {1, 2, 4}) {
    if (nr > 1 && nr > nsrc) continue;
    cand.nr = nr;
    cand.ct = 0;
    for (int bs : {64, 128, 256})
      for (int xcd : {0, 1}) {
        cand.bs = bs;
        cand.xcd = xcd;
        try_shape(cand);
      }
    cand.xcd = 1;
    if (nr <= 2) {
      cand.ct = -1;
      try_shape(cand);
    }
    for (int ct : {2, 4, 8, 16})
      for (int tbs = 64; tbs <= 1024; tbs += 64) {
        cand.ct = ct;
        cand.tbs = tbs;
        try_shape(cand);
      }
  }
  const Tune best = refine_shapes(trials, c->tune, [&](const Tune &cd) { return time_shape(cd, 10); });
  if (getenv("SSCG_VERBOSE"))
    fprintf(stderr, "[sscg] tuned %s: nr=%d bs=%d xcd=%d ct=%d tbs=%d\n", key.c_str(), best.nr, best.bs, best.xcd,
            best.ct, best.tbs);
  c->tuned[key] = best;
  return best;
}


static int host_sum_partials(sscg_ctx *c, const double *dev_partial, int nvec, int nblk, std::vector<double> &out,
                             hipStream_t st) {
  std::vector<double> h((size_t)nvec * nblk);
  HIPCHK(c, hipMemcpyAsync(h.data(), dev_partial, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  out.assign(nvec, 0.0);
  for (int v = 0; v < nvec; ++v)
    for (int b = 0; b < nblk; ++b) out[v] += h[(size_t)v * nblk + b];
  return SSCG_OK;
}

// Order the private stream after the caller's stream.
static int join_user(sscg_ctx *c) {
  HIPCHK(c, hipEventRecord(c->ev_sync, c->user));
  HIPCHK(c, hipStreamWaitEvent(c->work, c->ev_sync, 0));
  return SSCG_OK;
}

// ---------------------------------------------------------------------------
// shifted CG over one or several problems

struct Prob {
  sscg_ctx *c = nullptr;
  const void *v = nullptr;  // canonical device
  int L = 0, N = 0;
  double sigma = 0.0;
  std::vector<double> z;    // 2N
  void *y = nullptr;        // device [L][N][n]: planar FP64 during the solve
  bool keep_planar = false; // leave y planar (internal callers)
  int32_t *conv_iter = nullptr;
  double *true_res = nullptr;
  int32_t *iters = nullptr;
  int status = SSCG_OK;
  int switch_iter = -1;   // iteration at which the FP32 phase began (output)
  double max_true_res = -1.0;  // largest FP64 true residual if computed (output), else -1
  // moments accumulated inside the solve (y == nullptr then): S device FP64
  // planar [nmom][L][n] (zeroed by the caller), coefficients device [nmom][N]
  void *mom = nullptr;
  const void *mom_coef = nullptr;
  int nmom = 0;
  int blk = 0;  // block length of the in-loop update's block form (0: per iteration)
  std::vector<double> tscale;  // per-shift tolerance multipliers (empty: all 1)
};

struct IterPlan {
  DslashBatch d64, d32, dru;
  ScalarBatch alpha;
  VecBatch r64, r32, u64, u32, u32s, fold_seed, rel;
  VecBatch m64, m32;  // shift update with in-loop moments (FP64 / FP32 shift vectors)
  VecBatch mt;        // its table kernel (per (source, shift) scalars of the iteration)
  VecBatch sp, bc;    // block form: seed direction update, composition of a block
  int blk;            // block form: block length (0: the per-iteration form)
  int nmom_max;       // 0: the solutions are stored
  int mom_ub;         // shifts per load batch of the in-loop moment update
  int mom_pf;         // in-loop moment update: next batch's loads issued before this batch's stores
  int ct;             // dslash kernel: t-slices per block (0: site-parallel)
  bool fuse_alpha;    // the residual update forms the seed step length itself
};
constexpr int kFuseAlphaMax = 1024;  // <p, Bp> partials per source up to which the step length is fused

static void build_plan(std::vector<Prob> &P, IterPlan &pl, const sscg_solve_opts &o, const Tune &t) {
  memset(&pl, 0, sizeof(pl));
  int bd = 0, bdru = 0, bs = 0, bv = 0, bu = 0, bm = 0, bmt = 0, bbc = 0;
  // one shift per group, the next shift's loads ahead of this shift's stores: the
  // fastest form at 24^3 x 48 in FP64 and with FP32 directions
  pl.mom_ub = env_int("SSCG_MOMUB", 1);
  pl.mom_pf = env_int("SSCG_MOMPF", 1);
  const int np = (int)P.size();
  pl.blk = P[0].blk;  // one form per batch (run_solve sets it for every problem)
  // the tile kernel needs a tile of t.tbs sites on every lattice of the batch, with
  // LDS for FP64 spinors (the FP64 phase and the reliable updates use it too)
  pl.ct = t.ct;
  // small lattices: the seed step length is formed inside the residual update from
  // the few <p, Bp> partials (one launch less per iteration)
  pl.fuse_alpha = env_int("SSCG_FUSE_ALPHA", 1) != 0;
  for (int i = 0; i < np; ++i)
    if ((P[i].c->V + 63) / 64 > kFuseAlphaMax) pl.fuse_alpha = false;
  std::vector<int> tys(np, 0), tzs(np, 0);
  for (int i = 0; i < np; ++i)
    if (pl.ct > 0 && !tile_shape(P[i].c, t.tbs, t.nr, 0, tys[i], tzs[i])) pl.ct = 0;
  if (pl.ct < 0 && t.nr > 2) pl.ct = 0;
  for (int i = 0; i < np; ++i) {
    sscg_ctx *c = P[i].c;
    const int L = P[i].L, N = P[i].N;
    const int nbs = nblk_site(c, t.bs, pl.ct, tys[i], tzs[i]), nbv = nblk_vec(c);
    const int nbr = std::min(nbv, kMaxRR);
    const int groups = (L + t.nr - 1) / t.nr;
    SeedState *seed = (SeedState *)c->seed.p;
    ShiftState *shift = (ShiftState *)c->shift.p;
    auto mk_d = [&](DslashJob &j, const void *in, void *out, const void *g, double *part, int begin) {
      j.in = in; j.out = out; j.gauge = g; j.partial = part; j.seed = seed;
      j.kappa = c->kappa; j.sigma = P[i].sigma;
      for (int k = 0; k < 4; ++k) j.dims[k] = c->dims[k];
      j.V = c->V; j.nsrc = L; j.nblk_site = nbs; j.block_begin = begin; j.nblocks = nbs * groups; j.mode = 1;
      j.ct = pl.ct;
      j.ty = tys[i];
      j.tz = tzs[i];
      j.order = c->dorder;
    };
    mk_d(pl.d64.job[i], c->p64.p, c->q64.p, c->g64.p, (double *)c->pq_part.p, bd);
    mk_d(pl.d32.job[i], c->p32.p, c->q32.p, c->g32.p, (double *)c->pq_part.p, bd);
    mk_d(pl.dru.job[i], c->xpart64.p, c->q64.p, c->g64.p, nullptr, bdru);
    // the iteration's first launch commits the staged state of the previous one
    for (DslashJob *dj : {&pl.d64.job[i], &pl.d32.job[i]}) {
      dj->shift = shift;
      dj->nshift = N;
    }
    bd += nbs * groups;
    bdru += nbs * groups;
    {
      ScalarJob &j = pl.alpha.job[i];
      j.seed = seed;
      j.partial = (const double *)c->pq_part.p;
      j.nblk = (c->V + 63) / 64;
      j.nsrc = L;
      j.block_begin = bs;
    }
    bs += L;
    auto mk_v = [&](VecJob &j, void *a, void *b, void *cc, void *d, int begin, int nblocks) {
      j.a = a; j.b = b; j.c = cc; j.d = d; j.e = nullptr; j.partial = (double *)c->rr_part.p;
      j.seed = seed; j.shift = shift; j.n = c->n; j.nsrc = L; j.nshift = N; j.nblk_vec = nbv;
      j.block_begin = begin; j.nblocks = nblocks; j.wbatch = t.wbatch; j.border = t.border;
      j.rr_partial = (const double *)c->rr_part.p; j.nrr = nbr; j.tol = o.tol;
    };
    // the seed passes run at most kMaxRR blocks per source (strided over the
    // entries), so the <r, r> partials every shift-update block sums stay few
    auto seed_pass = [&](VecJob &j, void *a, void *b, void *cc, void *d) {
      mk_v(j, a, b, cc, d, bv, L * nbr);
      j.nblk_vec = nbr;
    };
    seed_pass(pl.r64.job[i], pl.blk > 0 ? c->ring.p : c->r64.p, c->q64.p, nullptr, nullptr);
    if (pl.blk > 0) {
      pl.r64.job[i].ring = pl.blk;
      seed_pass(pl.sp.job[i], c->ring.p, nullptr, nullptr, c->p64.p);
      pl.sp.job[i].ring = pl.blk;
    }
    seed_pass(pl.r32.job[i], c->r32.p, c->q32.p, c->xpart32.p, c->p32.p);
    if (pl.fuse_alpha)
      for (VecJob *rj : {&pl.r64.job[i], &pl.r32.job[i]}) {
        rj->npq = (c->V + 63) / 64;
        rj->pq_partial = (const double *)c->pq_part.p;
      }
    seed_pass(pl.fold_seed.job[i], c->xpart64.p, c->xpart32.p, nullptr, nullptr);
    seed_pass(pl.rel.job[i], c->rbase.p, c->q64.p, c->r64.p, c->r32.p);
    bv += L * nbr;
    const int nbatch = (N + t.wbatch - 1) / t.wbatch;
    mk_v(pl.u64.job[i], P[i].y, c->W.p, c->r64.p, c->p64.p, bu, L * nbatch * nbv);
    mk_v(pl.u32.job[i], P[i].y, c->W.p, c->r32.p, c->p32.p, bu, L * nbatch * nbv);
    mk_v(pl.u32s.job[i], P[i].y, c->W.p, c->r64.p, c->p64.p, bu, L * nbatch * nbv);
    bu += L * nbatch * nbv;
    if (P[i].nmom > 0) {
      const int nbm = (int)((c->n + kMomBlock - 1) / kMomBlock);
      for (VecBatch *mb : {&pl.m64, &pl.m32}) {
        VecJob &j = mb->job[i];
        mk_v(j, P[i].mom, c->W.p, pl.blk > 0 ? c->ring.p : c->r64.p, pl.blk > 0 ? c->v64.p : c->p64.p, bm,
             L * nbm);
        j.e = c->momtab.p;
        j.ring = pl.blk;
        j.mcoef = (const double2 *)P[i].mom_coef;
        j.nmom = P[i].nmom;
        j.nblk_mom = nbm;
      }
      bm += L * nbm;
      const int nch = (N + kBlock - 1) / kBlock;
      VecJob &jt = pl.mt.job[i];
      mk_v(jt, P[i].mom, c->W.p, c->r64.p, c->p64.p, bmt, L * nch);
      jt.e = c->momtab.p;
      jt.mcoef = (const double2 *)P[i].mom_coef;
      jt.nmom = P[i].nmom;
      jt.ring = pl.blk;
      bmt += L * nch;
      if (pl.blk > 0) {  // composition: one block per source
        VecJob &jc = pl.bc.job[i];
        mk_v(jc, P[i].mom, c->W.p, c->ring.p, c->p64.p, bbc, L);
        jc.e = c->momtab.p;
        jc.mcoef = (const double2 *)P[i].mom_coef;
        jc.nmom = P[i].nmom;
        jc.ring = pl.blk;
        bbc += L;
      }
      pl.nmom_max = std::max(pl.nmom_max, P[i].nmom);
    }
  }
  pl.m64.njobs = pl.m32.njobs = pl.mt.njobs = np;
  pl.m64.total_blocks = pl.m32.total_blocks = bm;
  pl.mt.total_blocks = bmt;
  pl.bc.njobs = pl.blk > 0 ? np : 0;
  pl.bc.total_blocks = bbc;
  pl.d64.njobs = pl.d32.njobs = pl.dru.njobs = np;
  pl.d64.commit = pl.d32.commit = 1;  // the iteration's first launch commits the previous one
  pl.d64.total_blocks = pl.d32.total_blocks = bd;
  pl.dru.total_blocks = bdru;
  pl.alpha.njobs = np;
  pl.alpha.total_blocks = bs;
  for (VecBatch *vb : {&pl.r64, &pl.r32, &pl.fold_seed, &pl.rel}) {
    vb->njobs = np;
    vb->total_blocks = bv;
  }
  pl.sp.njobs = pl.blk > 0 ? np : 0;
  pl.sp.total_blocks = pl.blk > 0 ? bv : 0;
  pl.u64.njobs = pl.u32.njobs = pl.u32s.njobs = np;
  pl.u64.total_blocks = pl.u32.total_blocks = pl.u32s.total_blocks = bu;
}

// Per-stage timing with HIP events on the solver stream: an event is recorded
// before each stage launch (or, sampled, around two of them) and the intervals
// are read at the next poll. Inside a captured graph the marks are event-record
// nodes, so the same events are rewritten by every replay and read after it; the
// marks of direct launches are read and cleared at every poll.
struct Recorder {
  sscg_ctx *c;
  hipStream_t st;
  bool on;
  std::vector<int> stages;
  std::vector<hipEvent_t> *evs;  // event pool (nullptr: the context's)
  bool in_graph = false;
  std::vector<int> its;  // iteration (in the chunk) of each mark
  int cur_it = 0;        // iteration the next marks belong to
  std::vector<hipEvent_t> &pool() { return evs ? *evs : c->events; }
  // event-record node appended to the capture by hand (after the nodes captured so
  // far; the next captured launch depends on it)
  hipError_t record_node(hipEvent_t e) {
    hipStreamCaptureStatus cs;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    hipError_t r = hipStreamGetCaptureInfo_v2(st, &cs, nullptr, &g, &deps, &nd);
    if (r != hipSuccess) return r;
    if (cs != hipStreamCaptureStatusActive || !g) return hipErrorIllegalState;
    hipGraphNode_t node = nullptr;
    r = hipGraphAddEventRecordNode(&node, g, deps, nd, e);
    if (r != hipSuccess) return r;
    return hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies);
  }
  void mark(int stage) {
    if (!on) return;
    const size_t k = stages.size();
    std::vector<hipEvent_t> &ev = pool();
    if (k >= ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        (void)hipGetLastError();
        return;
      }
      ev.push_back(e);
    }
    const hipError_t r = in_graph ? record_node(ev[k]) : hipEventRecord(ev[k], st);
    if (r != hipSuccess) {
      on = false;  // timing is best effort; never leave a sticky error behind
      (void)hipGetLastError();
      fprintf(stderr, "sscg: stage timing off (%s event record: %s)\n", in_graph ? "graph" : "stream",
              hipGetErrorString(r));
      return;
    }
    stages.push_back(stage);
    its.push_back(cur_it);
  }
  // intervals between consecutive recorded events (all complete) -> stage totals;
  // an interval that starts at a stop mark (-1) is not counted, nor one of an
  // iteration k0 + it at or after kend (no source iterated any more: its launches
  // exit at once), nor a block sweep whose whole block lies there (blk: block length)
  void account(int64_t k0 = 0, int64_t kend = INT64_MAX, int blk = 0) {
    std::vector<hipEvent_t> &ev = pool();
    for (size_t k = 0; k + 1 < stages.size(); ++k) {
      if (stages[k] < 0) continue;
      const int64_t g = k0 + (k < its.size() ? its[k] : 0);
      if (stages[k] == ST_PASS ? g - blk + 1 >= kend : g >= kend) continue;
      float ms = 0.f;
      const hipError_t r = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      if (r != hipSuccess) {
        (void)hipGetLastError();
        fprintf(stderr, "sscg: stage timing off (elapsed time: %s)\n", hipGetErrorString(r));
        on = false;
        return;
      }
      c->stage_ms[stages[k]] += ms;
      c->stage_calls[stages[k]] += 1;
    }
  }
  void flush(int64_t k0 = 0, int64_t kend = INT64_MAX, int blk = 0) {
    if (!on || stages.empty()) return;
    mark(-1);
    hipEventSynchronize(pool()[stages.size() - 1]);
    account(k0, kend, blk);
    stages.clear();
    its.clear();
  }
};

// The iteration after its dslash: step length, seed residual, (reliable update,)
// shift update with the shift scalars. rec marks every stage; ru_rec (when given)
// brackets the reliable update alone.
static void launch_iteration_tail(const IterPlan &pl, int prec, bool seed32, bool ru, int lr, const Tune &t,
                                  hipStream_t st, Recorder &rec, Recorder *ru_rec, int slot) {
  const int sp = (prec == 1 && seed32) ? 1 : 0;  // seed precision
  if (!pl.fuse_alpha) {
    rec.mark(ST_ALPHA);
    launch_seed_alpha(pl.alpha, st);
  }
  rec.mark(ST_RUPD);
  const bool ru_now = sp == 1 && ru;
  launch_seed_r_update(sp == 0 ? pl.r64 : pl.r32, sp, st, slot);
  if (ru_now) {
    rec.mark(ST_RU);
    if (ru_rec) ru_rec->mark(ST_RU);
    launch_fold_seed(pl.fold_seed, st);
    launch_dslash(pl.dru, 0, t.nr, 18, t.bs, t.xcd, pl.ct, st);
    launch_reliable_residual(pl.rel, st);
    if (ru_rec) ru_rec->mark(-1);
  }
  rec.mark(ST_SHIFT);
  if (pl.nmom_max > 0 && pl.blk > 0) {  // block form: the sweep after a block's last iteration
    launch_shift_table(pl.mt, st, slot);
    launch_seed_p_update(pl.sp, slot, st);
    if (slot == pl.blk - 1) {
      rec.mark(ST_PASS);
      launch_blk_compose(pl.bc, pl.blk, prec, st);
      launch_blk_pass(prec == 0 ? pl.m64 : pl.m32, prec, pl.nmom_max, pl.blk, st);
    }
  } else if (pl.nmom_max > 0) {  // FP64 seed in both phases (checked by run_solve)
    launch_shift_table(pl.mt, st);
    launch_shift_moments_tab(prec == 0 ? pl.m64 : pl.m32, prec, pl.nmom_max, pl.mom_ub, pl.mom_pf, st);
  } else {
    const VecBatch &u = prec == 0 ? pl.u64 : (sp == 1 ? pl.u32 : pl.u32s);
    launch_shift_update(u, prec, sp, prec == 1 && ru, t.unroll, t.nt, st);
  }
}

// One iteration. prec: 0 FP64 phase, 1 FP32 phase; seed32: the FP32 phase also runs
// the seed in FP32 (SSCG_MIXED) rather than FP64 (SSCG_MIXED_SHIFTS); ru: last
// iteration of an FP32 chunk (seed reliable update if seed32, fold of the FP32
// shift partials into the FP64 solutions in both FP32 modes).
// Timing marks: with every == 1 each launch is bracketed (the marks chain, one
// interval per stage); with every == k > 1 every stage of the iterations
// it % k == k / 2 is bracketed (a chain of marks closed by a stop mark; the first
// iteration after a poll, whose launches start on an idle device, is not sampled),
// and so is every reliable update (it falls on the last iteration of a chunk).
static void launch_iteration(const IterPlan &pl, int prec, bool seed32, bool ru, int lr, const Tune &t,
                             hipStream_t st, Recorder &rec, int it = 0, int every = 1) {
  const int sp = (prec == 1 && seed32) ? 1 : 0;  // seed precision
  // block form: chunks start at multiples of the block length, so the iteration's
  // place in its block is its place in the chunk modulo the block length
  const int slot = pl.blk > 0 ? it % pl.blk : 0;
  if (every > 1) {
    // block form: the sampled iterations are last iterations of a block (about one in
    // every), so the block sweep is timed with the rest
    const int q = pl.blk > 0 ? std::max(1, every / pl.blk) : 1;
    const bool smp = pl.blk > 0 ? (slot == pl.blk - 1 && (it / pl.blk) % q == q / 2) : it % every == every / 2;
    Recorder off{rec.c, st, false, {}, nullptr};
    Recorder &r = smp ? rec : off;
    rec.cur_it = it;
    r.mark(ST_DSLASH);
    launch_dslash(sp == 0 ? pl.d64 : pl.d32, sp, t.nr, sp == 0 ? 18 : lr, t.bs, t.xcd, pl.ct, st);
    launch_iteration_tail(pl, prec, seed32, ru, lr, t, st, r, smp ? nullptr : &rec, slot);
    r.mark(-1);
    return;
  }
  rec.cur_it = it;
  rec.mark(ST_DSLASH);
  launch_dslash(sp == 0 ? pl.d64 : pl.d32, sp, t.nr, sp == 0 ? 18 : lr, t.bs, t.xcd, pl.ct, st);
  launch_iteration_tail(pl, prec, seed32, ru, lr, t, st, rec, nullptr, slot);
}

static int prepare_problem(Prob &p, const sscg_solve_opts &o) {
  sscg_ctx *c = p.c;
  const size_t n = c->n, L = p.L, N = p.N;
  const size_t vec64 = n * sizeof(double2), vec32 = n * sizeof(float2);
  CHK(ensure(c, c->v64, L * vec64));
  CHK(ensure(c, c->r64, L * vec64));
  CHK(ensure(c, c->p64, L * vec64));
  CHK(ensure(c, c->q64, L * vec64));
  // shift directions: one vector per (source, shift), chunk-blocked and padded to a
  // multiple of 64 entries in the in-loop moment form
  const size_t npad = (n + 63) / 64 * 64;
  CHK(ensure(c, c->W, L * N * (p.nmom > 0 ? npad : n) * sizeof(double2)));
  CHK(ensure(c, c->tmp, vec64));
  CHK(ensure(c, c->pq_part, L * (size_t)((c->V + 63) / 64) * sizeof(double)));
  CHK(ensure(c, c->rr_part, std::max<size_t>(L * nblk_vec(c), L * 64) * sizeof(double)));
  CHK(ensure(c, c->seed, L * sizeof(SeedState)));
  CHK(ensure(c, c->shift, L * N * sizeof(ShiftState)));
  CHK(ensure(c, c->zdev, N * 2 * sizeof(double)));
  if (p.nmom > 0)
    CHK(ensure(c, c->momtab,
               p.blk > 0 ? blk_layout((int)L, (int)N, p.blk).total : shift_table_bytes((int)L, (int)N)));
  if (p.blk > 0) CHK(ensure(c, c->ring, (size_t)p.blk * L * vec64));
  if (o.prec == SSCG_MIXED) {  // FP32 seed vectors and reliable-update storage
    CHK(ensure(c, c->r32, L * vec32));
    CHK(ensure(c, c->p32, L * vec32));
    CHK(ensure(c, c->q32, L * vec32));
    CHK(ensure(c, c->rbase, L * vec64));
    CHK(ensure(c, c->xpart64, L * vec64));
    CHK(ensure(c, c->xpart32, L * vec32));
  }
  if (c->seed_host_cap < (int)L) {
    if (c->seed_host) hipHostFree(c->seed_host);
    c->seed_host = nullptr;
    if (hipHostMalloc((void **)&c->seed_host, L * sizeof(SeedState), hipHostMallocDefault) != hipSuccess)
      return fail(c, SSCG_ENOMEM, "pinned host allocation failed");
    c->seed_host_cap = (int)L;
  }
  hipStream_t st = c->work;
  // v -> planar FP64; r = p = v; p_j = v; x_j = 0
  launch_pack(p.v, c->v64.p, 0, (int)L, c->V, st);
  HIPCHK(c, hipMemcpyAsync(c->r64.p, c->v64.p, L * vec64, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->p64.p, c->v64.p, L * vec64, hipMemcpyDeviceToDevice, st));
  if (p.blk > 0) {
    // block form: r_0 = v in the ring's last slot, the other slots zero (a block cut
    // short reads slots it never wrote, with zero coefficients); history: identity
    HIPCHK(c, hipMemsetAsync(c->ring.p, 0, (size_t)(p.blk - 1) * L * vec64, st));
    HIPCHK(c, hipMemcpyAsync((char *)c->ring.p + (size_t)(p.blk - 1) * L * vec64, c->v64.p, L * vec64,
                             hipMemcpyDeviceToDevice, st));
    launch_blk_init(c->momtab.p, (int)L, (int)N, p.blk, st);
  }
  if (p.nmom == 0)
    launch_init_shifts(p.y, c->W.p, c->v64.p, (int64_t)n, (int)L, (int)N, st);
  else if (p.blk == 0)  // (the block form's first sweep reads v itself)
    launch_init_shifts_blocked(c->W.p, c->v64.p, (int64_t)n, (int)L, (int)N, st);
  // ||v||
  const int nb = 64;
  launch_norm2_partial(c->v64.p, c->n, (int)L, (double *)c->rr_part.p, nb, st);
  std::vector<double> vn2;
  CHK(host_sum_partials(c, (double *)c->rr_part.p, (int)L, nb, vn2, st));
  std::vector<SeedState> seeds(L);
  for (size_t l = 0; l < L; ++l) {
    if (!(vn2[l] > 0.0) || !std::isfinite(vn2[l]))
      return fail(c, SSCG_EINVAL, "source " + std::to_string(l) + " is zero or not finite");
    SeedState &s = seeds[l];
    memset(&s, 0, sizeof(s));
    s.rho = vn2[l];
    s.alpha_prev = 1.0;
    s.beta_prev = 0.0;
    s.vnorm = std::sqrt(vn2[l]);
    s.maxres = 1.0;
    s.nactive = (int)N;
    s.maxiter = o.maxiter;
  }
  std::vector<ShiftState> sh(L * N);
  for (size_t l = 0; l < L; ++l)
    for (size_t j = 0; j < N; ++j) {
      ShiftState &h = sh[l * N + j];
      memset(&h, 0, sizeof(h));
      h.s = make_double2(p.z[2 * j] - p.sigma, p.z[2 * j + 1]);
      h.pi_prev = h.pi_cur = make_double2(1.0, 0.0);
      h.active = 1;
      h.conv_iter = -1;
      h.tscale = p.tscale.empty() ? 1.0 : p.tscale[j];
    }
  HIPCHK(c, hipMemcpyAsync(c->seed.p, seeds.data(), L * sizeof(SeedState), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->shift.p, sh.data(), L * N * sizeof(ShiftState), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->zdev.p, p.z.data(), N * 2 * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipStreamSynchronize(st));
  return SSCG_OK;
}

// FP64 -> FP32 switch of one problem: seed vectors, reliable-update base, and the
// shift directions p_j (rewritten in place through one temporary vector).
static int switch_to_fp32(Prob &p, bool seed32, hipStream_t st) {
  sscg_ctx *c = p.c;
  const size_t n = c->n, L = p.L, N = p.N, vec64 = n * sizeof(double2);
  if (seed32) {
    launch_cast(c->r64.p, 0, c->r32.p, 1, (int64_t)(L * n), st);
    launch_cast(c->p64.p, 0, c->p32.p, 1, (int64_t)(L * n), st);
    HIPCHK(c, hipMemcpyAsync(c->rbase.p, c->r64.p, L * vec64, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemsetAsync(c->xpart64.p, 0, L * vec64, st));
    HIPCHK(c, hipMemsetAsync(c->xpart32.p, 0, L * n * sizeof(float2), st));
  }
  if (p.nmom > 0) {  // in-loop moment form: chunk-blocked directions, converted in place
    launch_blocked_to_fp32(c->W.p, (int64_t)n, (int)L, (int)N, st);
    return SSCG_OK;
  }
  for (size_t k = 0; k < L * N; ++k) {
    char *slot = (char *)c->W.p + k * vec64;
    HIPCHK(c, hipMemcpyAsync(c->tmp.p, slot, vec64, hipMemcpyDeviceToDevice, st));
    launch_to_fp32(c->tmp.p, slot, slot + n * sizeof(float2), (int64_t)n, st);
  }
  return SSCG_OK;
}

// Launch-shape autotuner. Times the dslash over (sources per thread, sites per
// block, XCD order) and the fused shift update over the shift-batch width on the
// problem's own buffers, before the first iteration. The shift update is timed
// as an identity (alpha_j = 0, beta_j = 1, 1/pi_j = 0 leaves x_j and p_j exactly
// as they are, and the seed p = r + 0 p = v is unchanged at the start), after
// which the initial solver state is uploaded again. Results are cached per shape.
static std::string tune_key(const std::vector<Prob> &P, const sscg_solve_opts &o) {
  std::string k = std::to_string(o.prec);
  for (const Prob &p : P)
    k += "|" + std::to_string(p.c->dims[0]) + "x" + std::to_string(p.c->dims[1]) + "x" +
         std::to_string(p.c->dims[2]) + "x" + std::to_string(p.c->dims[3]) + ":" + std::to_string(p.L) + ":" +
         std::to_string(p.N);
  return k;
}

static int autotune(std::vector<Prob> &P, const sscg_solve_opts &o, int lr, hipStream_t st, Tune &best) {
  sscg_ctx *c0 = P[0].c;
  const std::string key = tune_key(P, o);
  auto it = c0->tuned.find(key);
  if (it != c0->tuned.end()) {
    best = it->second;
    return SSCG_OK;
  }
  hipEvent_t e0, e1;
  HIPCHK(c0, hipEventCreate(&e0));
  HIPCHK(c0, hipEventCreate(&e1));
  auto time_it = [&](auto &&launch, int reps) -> double { return time_with_events(st, e0, e1, launch, reps); };
  int maxL = 1, maxN = 1;
  for (Prob &p : P) {
    maxL = std::max(maxL, p.L);
    maxN = std::max(maxN, p.N);
  }
  // dslash on the seed buffers (p -> q) in the precision most iterations use (FP32
  // when the seed switches to FP32, then on a copy of p); its partials are
  // rewritten by the first iteration
  const int dprec = o.prec == SSCG_MIXED ? 1 : 0;
  if (dprec == 1)
    for (Prob &p : P) launch_cast(p.c->p64.p, 0, p.c->p32.p, 1, (int64_t)p.L * p.c->n, st);
  Tune cand = best;
  std::vector<Trial> trials;
  auto time_shape = [&](const Tune &cd, int reps) {
    IterPlan pl;
    build_plan(P, pl, o, cd);
    return time_it([&] {
      launch_dslash(dprec ? pl.d32 : pl.d64, dprec, cd.nr, dprec ? lr : 18, cd.bs, cd.xcd, pl.ct, st);
    }, reps);
  };
  // site-parallel kernel: sources per thread, sites per block, XCD order
  auto try_shape = [&](const Tune &cd) {
    IterPlan pl;
    build_plan(P, pl, o, cd);
    if (cd.ct != 0 && pl.ct == 0) return;  // no tile of this size on some lattice
    trials.push_back({time_shape(cd, 5), (int)trials.size(), cd});
  };
  for (int nr : {1, 2, 4}) {
    if (nr > 1 && nr > maxL) continue;
    cand.nr = nr;
    cand.ct = 0;
    for (int bs : {64, 128, 256})
      for (int xcd : {0, 1}) {
        cand.bs = bs;
        cand.xcd = xcd;
        try_shape(cand);
      }
    // direction-split kernel (small lattices)
    cand.xcd = 1;
    if (nr <= 2) {
      cand.ct = -1;
      try_shape(cand);
    }
    // tile kernel: t-slices per block and tile size
    for (int ct : {2, 4, 8, 16})
      for (int tbs = 64; tbs <= 1024; tbs += 64) {
        cand.ct = ct;
        cand.tbs = tbs;
        try_shape(cand);
      }
  }
  {
    const Tune d = refine_shapes(trials, best, [&](const Tune &cd) { return time_shape(cd, 15); });
    best.nr = d.nr;
    best.bs = d.bs;
    best.xcd = d.xcd;
    best.ct = d.ct;
    best.tbs = d.tbs;
  }
  // fused shift update as an identity on the current data (identity jobs: every
  // shift updated with alpha_j = 0, beta_j = 1, 1/pi_j = 0, no state written; not
  // used, and not timed, when the moments are accumulated in the loop: there is no y_j)
  const bool tune_update = P[0].nmom == 0;
  for (Prob &p : P) {
    if (!tune_update) break;
    std::vector<SeedState> sd(p.L);
    HIPCHK(p.c, hipMemcpy(sd.data(), p.c->seed.p, sd.size() * sizeof(SeedState), hipMemcpyDeviceToHost));
    for (SeedState &x : sd) x.pending = 1;
    HIPCHK(p.c, hipMemcpy(p.c->seed.p, sd.data(), sd.size() * sizeof(SeedState), hipMemcpyHostToDevice));
  }
  cand = best;
  std::vector<Trial> utrials;
  auto time_update = [&](const Tune &cd, int reps) {
    IterPlan pl;
    build_plan(P, pl, o, cd);
    for (int i = 0; i < pl.u64.njobs; ++i) pl.u64.job[i].identity = 1;
    return time_it([&] { launch_shift_update(pl.u64, 0, 0, 0, cd.unroll, cd.nt, st); }, reps);
  };
  for (int w : {2, 4, 8, 16, 32}) {
    if (!tune_update) break;
    if (w > 2 && w / 2 >= maxN) continue;
    for (int u : {1, 2, 4}) {
      if (u > w) continue;
      for (int nt : {0, 1})
        for (int bo : {0, 1}) {
          cand.wbatch = w;
          cand.unroll = u;
          cand.nt = nt;
          cand.border = bo;
          utrials.push_back({time_update(cand, 3), (int)utrials.size(), cand});
        }
    }
  }
  if (tune_update) {
    const Tune d = refine_shapes(utrials, best, [&](const Tune &cd) { return time_update(cd, 10); });
    best.wbatch = d.wbatch;
    best.unroll = d.unroll;
    best.nt = d.nt;
    best.border = d.border;
  }
  if (getenv("SSCG_VERBOSE"))
    fprintf(stderr, "[sscg] tuned %s: nr=%d bs=%d xcd=%d ct=%d tbs=%d wbatch=%d unroll=%d nt=%d border=%d\n",
            key.c_str(), best.nr, best.bs, best.xcd, best.ct, best.tbs, best.wbatch, best.unroll, best.nt, best.border);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // restore the initial state
  for (Prob &p : P) {
    std::vector<SeedState> sd(p.L);
    HIPCHK(p.c, hipMemcpy(sd.data(), p.c->seed.p, sd.size() * sizeof(SeedState), hipMemcpyDeviceToHost));
    for (SeedState &x : sd) x.pending = 0;
    HIPCHK(p.c, hipMemcpy(p.c->seed.p, sd.data(), sd.size() * sizeof(SeedState), hipMemcpyHostToDevice));
  }
  c0->tuned[key] = best;
  return SSCG_OK;
}

static int run_solve(std::vector<Prob> &P, const sscg_solve_opts &o_in) {
  sscg_solve_opts o = o_in;
  if (o.poll_every < 1) o.poll_every = 1;
  if (o.ru_interval < 1) o.ru_interval = 50;
  sscg_ctx *c0 = P[0].c;
  hipStream_t st = c0->work;
  // block form of the in-loop moment update: block length 4, 8, 16, 24 or 32 (0: per iteration)
  const int blk = env_int("SSCG_BLOCK", 24);
  if (blk != 0 && blk != 4 && blk != 8 && blk != 16 && blk != 24 && blk != 32)
    return fail(c0, SSCG_EINVAL, "SSCG_BLOCK must be 0, 4, 8, 16, 24 or 32");
  for (Prob &p : P) p.blk = p.nmom > 0 ? blk : 0;
  for (Prob &p : P) {
    if (!p.c->have_gauge) return fail(p.c, SSCG_ESTATE, "no gauge field set");
    if (p.c->device != c0->device) return fail(c0, SSCG_EINVAL, "all problems must share one device");
    HIPCHK(p.c, hipSetDevice(p.c->device));
    CHK(join_user(p.c));
    CHK(prepare_problem(p, o));
  }
  if (P.size() > (size_t)kMaxJobs) return fail(c0, SSCG_EINVAL, "too many problems in one batch");
  // all problems' work goes to the first context's private stream
  for (Prob &p : P) {
    if (p.c != c0) {
      HIPCHK(p.c, hipEventRecord(p.c->ev_sync, p.c->work));
      HIPCHK(c0, hipStreamWaitEvent(st, p.c->ev_sync, 0));
    }
  }
  for (Prob &p : P)
    if ((p.nmom > 0) != (P[0].nmom > 0) || (p.nmom > 0 && (o.prec == SSCG_MIXED || p.nmom > 32 || !p.mom)))
      return fail(c0, SSCG_EINVAL, "in-loop moments need an FP64 seed, at most 32 moments, and one mode per batch");
  int lr = 18;
  for (Prob &p : P) lr = std::min(lr, p.c->link_reals);
  for (Prob &p : P)
    if (p.c->link_reals != lr) return fail(c0, SSCG_EINVAL, "all problems of a batch must use one link format");
  Tune tn = c0->tune;
  if (c0->autotune) {
    CHK(autotune(P, o, lr, st, tn));
  }
  IterPlan pl;
  build_plan(P, pl, o, tn);
  for (int i = 0; i < ST_N; ++i) {
    c0->stage_ms[i] = 0.0;
    c0->stage_calls[i] = 0;
    c0->stage_launched[i] = 0;
  }
  // launches of each stage in a chunk of len iterations of phase prec
  auto count_chunk = [&](int prec, int len, bool full) {
    int64_t *n = c0->stage_launched;
    n[ST_DSLASH] += len;
    n[ST_RUPD] += len;
    n[ST_SHIFT] += len;
    if (!pl.fuse_alpha) n[ST_ALPHA] += len;
    if (prec == 1 && o.prec == SSCG_MIXED && full) n[ST_RU] += 1;
    if (pl.blk > 0) n[ST_PASS] += len / pl.blk;
  };
  Recorder rec{c0, st, c0->profiling > 0, {}, nullptr};
  // profiling level 1 times every launch and runs them directly (an event-record node
  // in a graph costs more than the launch gap it would hide); a level k > 1 samples
  // every k-th iteration and keeps graph replay
  const int every = c0->profiling > 1 ? c0->profiling : 1;
  const bool use_graph = o.use_graph != 0 && c0->profiling != 1;
  const bool seed32 = o.prec == SSCG_MIXED;
  // timing marks of the graphs: events owned by the context, rewritten by each replay
  Recorder grec[2] = {{c0, st, false, {}, &c0->graphs[0].ev}, {c0, st, false, {}, &c0->graphs[1].ev}};
  // everything a captured chunk depends on: the launch plan (kernel arguments and
  // buffer addresses), the launch shapes, the phase, the length, the timing level
  auto graph_key = [&](int prec, int len) {
    std::string key(reinterpret_cast<const char *>(&pl), sizeof(pl));
    const int64_t v[] = {prec, len, lr, every, c0->profiling, seed32 ? 1 : 0, tn.nr, tn.bs, tn.wbatch, tn.xcd,
                         tn.unroll, tn.nt, tn.ct, tn.tbs, tn.border, (int64_t)(intptr_t)st};
    key.append(reinterpret_cast<const char *>(v), sizeof(v));
    return key;
  };
  auto capture = [&](int prec, int len) -> int {
    sscg_ctx::CachedGraph &cg = c0->graphs[prec];
    const std::string key = graph_key(prec, len);
    if (cg.exec && cg.key == key) {  // replay the graph of an earlier solve
      grec[prec].on = cg.timed;
      grec[prec].in_graph = true;
      grec[prec].stages = cg.stages;
      grec[prec].its = cg.its;
      return SSCG_OK;
    }
    if (cg.exec) hipGraphExecDestroy(cg.exec);
    cg.exec = nullptr;
    cg.key.clear();
    hipGraph_t g = nullptr;
    Recorder &cap = grec[prec];
    cap.on = c0->profiling > 0;
    cap.in_graph = true;
    cap.stages.clear();
    cap.its.clear();
    // events exist before capture; they only time, so they skip the system-scope
    // release (cache write-back) an event normally carries, which shortens the node
    while (cap.on && cg.ev.size() < (size_t)len * (ST_N + 1) + 1) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipGetLastError();
        cap.on = false;
        break;
      }
      cg.ev.push_back(e);
    }
    HIPCHK(c0, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < len; ++k)
      launch_iteration(pl, prec, seed32, prec == 1 && k == len - 1, lr, tn, st, cap, k, every);
    if (every == 1) cap.mark(-1);
    HIPCHK(c0, hipStreamEndCapture(st, &g));
    const hipError_t ie = hipGraphInstantiate(&cg.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      cg.exec = nullptr;
      return fail(c0, SSCG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    cg.key = key;
    cg.stages = cap.stages;
    cg.its = cap.its;
    cg.timed = cap.on;
    return SSCG_OK;
  };
  bool ready[2] = {false, false};  // graph of this phase checked against this solve
  int64_t kwork = 0;                // iterations in which a source still iterated
  auto t0 = std::chrono::steady_clock::now();
  int prec = 0;
  int k = 0;
  int rc = SSCG_OK;
  while (k < o.maxiter) {
    // the FP64 phase of a mixed solve polls at least every 10 iterations so the
    // switch to FP32 is not delayed by a long poll interval
    int period = prec == 1 ? o.ru_interval
                           : (o.prec != SSCG_FP64 ? std::min(o.poll_every, 10) : o.poll_every);
    if (pl.blk > 0) period = (period + pl.blk - 1) / pl.blk * pl.blk;  // polls at block ends
    const int chunk = std::min(period, o.maxiter - k);
    const bool full = chunk == period;
    if (use_graph && full) {
      if (!ready[prec]) {
        rc = capture(prec, chunk);
        if (rc != SSCG_OK) break;
        ready[prec] = true;
      }
      hipError_t e = hipGraphLaunch(c0->graphs[prec].exec, st);
      if (e != hipSuccess) {
        rc = fail(c0, SSCG_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        break;
      }
    } else {
      for (int kk = 0; kk < chunk; ++kk)
        launch_iteration(pl, prec, seed32, prec == 1 && (kk == chunk - 1) && full, lr, tn, st, rec, kk, every);
    }
    count_chunk(prec, chunk, full);
    k += chunk;
    // poll: commit the last iteration's staged state, then read the seed states
    if (!(use_graph && full)) rec.mark(-1);
    launch_commit(pl.d64, st);
    bool all_done = true, can_switch = true;
    for (Prob &p : P) {
      hipError_t e = hipMemcpyAsync(p.c->seed_host, p.c->seed.p, p.L * sizeof(SeedState),
                                    hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) {
        rc = fail(c0, SSCG_EDEVICE, "poll copy failed");
        break;
      }
    }
    if (rc != SSCG_OK) break;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rc = fail(c0, SSCG_EDEVICE, std::string("solve loop: ") + hipGetErrorString(e));
      break;
    }
    // iterations up to which a source still iterated: timing samples beyond are not
    // counted (their launches exit at once)
    for (Prob &p : P)
      for (int l = 0; l < p.L; ++l) kwork = std::max<int64_t>(kwork, p.c->seed_host[l].iters);
    rec.flush(k - chunk, kwork, pl.blk);
    if (use_graph && full && grec[prec].on) grec[prec].account(k - chunk, kwork, pl.blk);
    for (Prob &p : P)
      for (int l = 0; l < p.L; ++l) {
        const SeedState &s = p.c->seed_host[l];
        if (!s.done) {
          all_done = false;
          if (!(s.maxres < o.switch_tol)) can_switch = false;
        }
      }
    if (all_done) break;
    if (o.prec != SSCG_FP64 && prec == 0 && can_switch) {
      for (Prob &p : P) {
        rc = switch_to_fp32(p, seed32, st);
        if (rc != SSCG_OK) break;
      }
      if (rc != SSCG_OK) break;
      prec = 1;
      for (Prob &p : P) p.switch_iter = k;
    }
  }
  if (rc != SSCG_OK) return rc;
  // launches that did work: the per-iteration stages of the iterations in which a source
  // still iterated, the sweeps of blocks holding such iterations
  {
    int64_t *n = c0->stage_launched;
    for (int s : {(int)ST_DSLASH, (int)ST_ALPHA, (int)ST_RUPD, (int)ST_SHIFT}) n[s] = std::min<int64_t>(n[s], kwork);
    if (pl.blk > 0) n[ST_PASS] = (kwork + pl.blk - 1) / pl.blk;
  }
  if (pl.blk > 0) {
    // block form: a block cut short by the iteration limit is swept now (after a
    // complete block the history is the identity and the sweep returns at once)
    launch_blk_compose(pl.bc, pl.blk, prec, st);
    launch_blk_pass(prec == 0 ? pl.m64 : pl.m32, prec, pl.nmom_max, pl.blk, st);
  }
  launch_commit(pl.d64, st);  // (every chunk ends with a commit; kept for a loop left early)
  if (prec == 1) {
    // fold every shift's FP32 partial into its FP64 solution
    for (Prob &p : P)
      if (p.y) launch_fold_shifts(p.y, p.c->W.p, p.c->n, p.L * p.N, st);
  }
  HIPCHK(c0, hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  c0->stage_ms[ST_LOOP] = std::chrono::duration<double, std::milli>(t1 - t0).count();
  c0->stage_calls[ST_LOOP] = k;
  c0->stage_launched[ST_LOOP] = k;
  // results
  int worst = SSCG_OK;
  for (Prob &p : P) {
    sscg_ctx *c = p.c;
    const int L = p.L, N = p.N;
    c->sweep_bytes = 0;
    if (p.blk > 0) {
      // bytes the sweep kernels moved, from the counts the compose kernel kept: per
      // (source, block) run of the moment kernel the residuals and the moment sums
      // read and written, per run of the direction kernel the residuals; per direction
      // read or written its entries (16 B FP64, 8 B FP32)
      const BlkLayout lay = blk_layout(L, N, p.blk);
      unsigned long long cnt[2 * kBlkCnt];
      HIPCHK(c, hipMemcpy(cnt, (char *)c->momtab.p + lay.cnt, sizeof(cnt), hipMemcpyDeviceToHost));
      for (int ph = 0; ph < 2; ++ph) {
        const unsigned long long *k = cnt + ph * kBlkCnt;
        const int64_t d = ph == 0 ? 16 : 8;
        const int64_t per_entry = (int64_t)k[0] * (16 * p.blk + 32 * p.nmom) + (int64_t)k[1] * d +
                                  (int64_t)k[2] * 16 * p.blk + (int64_t)(k[3] + k[4]) * d;
        c->sweep_bytes += per_entry * c->n;
      }
    }
    std::vector<SeedState> seeds(L);
    std::vector<ShiftState> sh((size_t)L * N);
    HIPCHK(c, hipMemcpy(seeds.data(), c->seed.p, L * sizeof(SeedState), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(sh.data(), c->shift.p, (size_t)L * N * sizeof(ShiftState), hipMemcpyDeviceToHost));
    int st_p = SSCG_OK;
    for (int l = 0; l < L; ++l) {
      if (p.iters) p.iters[l] = seeds[l].iters;
      int s = seeds[l].done ? seeds[l].status : SSCG_ENOTCONV;
      if (s == SSCG_EBREAKDOWN) st_p = SSCG_EBREAKDOWN;
      else if (s == SSCG_ENOTCONV && st_p == SSCG_OK) st_p = SSCG_ENOTCONV;
      for (int j = 0; j < N; ++j)
        if (p.conv_iter) p.conv_iter[(size_t)l * N + j] = sh[(size_t)l * N + j].conv_iter;
    }
    // FP64 true residuals ||v - (z_j - A) y_j|| / ||v||: when the caller asks for them,
    // and always after a mixed-precision solve, whose FP32 updates can leave a shift's
    // true residual above the implicit one that froze it; such a solve returns
    // SSCG_EINACCURATE when one exceeds true_factor * tol (times the shift's own
    // tolerance multiplier)
    p.max_true_res = -1.0;
    const bool mixed = o.prec != SSCG_FP64;
    if (p.y && (p.true_res || mixed)) {
      const size_t n = c->n, vec64 = n * sizeof(double2);
      const int nb = 64;
      std::vector<double> local;
      double *tr = p.true_res;
      if (!tr) {
        local.resize((size_t)L * N);
        tr = local.data();
      }
      // A y_j for L shifts at a time into q64 (one dslash launch), then the residual
      // partials of those shifts; one read-back of all partials at the end
      CHK(ensure(c, c->trpart, (size_t)L * N * nb * sizeof(double)));
      double *part = (double *)c->trpart.p;
      for (int l = 0; l < L; ++l) {
        for (int j0 = 0; j0 < N; j0 += L) {
          const int cnt = std::min(L, N - j0);
          const char *yj = (const char *)p.y + ((size_t)l * N + j0) * vec64;
          dslash_with(c, apply_tune(c, yj, c->q64.p, cnt, 0, st), yj, c->q64.p, cnt, 0, 0, 0.0, nullptr, nullptr, st);
          launch_true_residual((const char *)c->v64.p + l * vec64, yj, c->q64.p, (const double *)c->zdev.p + 2 * j0,
                               (int64_t)n, cnt, part + ((size_t)l * N + j0) * nb, nb, st);
        }
      }
      std::vector<double> r2;
      CHK(host_sum_partials(c, part, L * N, nb, r2, st));
      for (int l = 0; l < L; ++l)
        for (int j = 0; j < N; ++j) tr[(size_t)l * N + j] = std::sqrt(r2[(size_t)l * N + j]) / seeds[l].vnorm;
      bool inaccurate = false;
      for (int l = 0; l < L; ++l)
        for (int j = 0; j < N; ++j) {
          const double t = tr[(size_t)l * N + j];
          p.max_true_res = std::max(p.max_true_res, t);
          const double scale = p.tscale.empty() ? 1.0 : p.tscale[j];
          if (!(t <= o.true_factor * o.tol * scale)) inaccurate = true;
        }
      if (mixed && o.true_factor > 0 && inaccurate && st_p == SSCG_OK) st_p = SSCG_EINACCURATE;
    }
    p.status = st_p;
    if (st_p == SSCG_EBREAKDOWN) worst = SSCG_EBREAKDOWN;
    else if (st_p == SSCG_ENOTCONV && worst != SSCG_EBREAKDOWN) worst = SSCG_ENOTCONV;
    else if (st_p == SSCG_EINACCURATE && worst == SSCG_OK) worst = SSCG_EINACCURATE;
    if (!p.keep_planar && p.y) {
      const size_t n = c->n, vec64 = n * sizeof(double2);
      for (size_t kk = 0; kk < (size_t)L * N; ++kk) {
        char *slot = (char *)p.y + kk * vec64;
        HIPCHK(c, hipMemcpyAsync(c->tmp.p, slot, vec64, hipMemcpyDeviceToDevice, st));
        launch_unpack(c->tmp.p, 0, slot, 1, c->V, st);
      }
    }
  }
  HIPCHK(c0, hipStreamSynchronize(st));
  return worst;
}

// ---------------------------------------------------------------------------
// quadrature (host, FP64)

extern "C" {

int sscg_quad_lines(int32_t N, double gamma, double rho, double beta, double *z, double *zeta, double *w) {
  if (N < 4 || N % 2 || !(rho > 0) || !(beta > 0)) return fail(nullptr, SSCG_EINVAL, "need even N >= 4, rho > 0, beta > 0");
  std::vector<cd> Z, ZE, W;
  quad_lines_host(N, gamma, rho, beta, Z, ZE, W);
  for (int j = 0; j < N; ++j) {
    if (z) { z[2 * j] = Z[j].real(); z[2 * j + 1] = Z[j].imag(); }
    if (zeta) { zeta[2 * j] = ZE[j].real(); zeta[2 * j + 1] = ZE[j].imag(); }
    if (w) { w[2 * j] = W[j].real(); w[2 * j + 1] = W[j].imag(); }
  }
  return SSCG_OK;
}

int sscg_quad_circle(int32_t N, double gamma, double rho, double *z, double *zeta, double *w) {
  if (N < 2 || !(rho > 0)) return fail(nullptr, SSCG_EINVAL, "need N >= 2, rho > 0");
  std::vector<cd> Z, ZE, W;
  quad_circle_host(N, gamma, rho, Z, ZE, W);
  for (int j = 0; j < N; ++j) {
    if (z) { z[2 * j] = Z[j].real(); z[2 * j + 1] = Z[j].imag(); }
    if (zeta) { zeta[2 * j] = ZE[j].real(); zeta[2 * j + 1] = ZE[j].imag(); }
    if (w) { w[2 * j] = W[j].real(); w[2 * j + 1] = W[j].imag(); }
  }
  return SSCG_OK;
}

int sscg_herm_eig(int32_t n, const double *A, double *evals, double *evecs) {
  if (n <= 0 || !A || !evals) return fail(nullptr, SSCG_EINVAL, "bad argument");
  if (!herm_eig(n, A, evals, evecs)) return fail(nullptr, SSCG_ENOTCONV, "QR iteration did not converge");
  return SSCG_OK;
}

int sscg_apply_A(sscg_ctx *c, const void *x, void *y, int32_t nsrc, int32_t prec) {
  if (!c || !x || !y || nsrc <= 0) return fail(c, SSCG_EINVAL, "bad argument");
  if (prec != SSCG_FP64 && prec != SSCG_MIXED) return fail(c, SSCG_EINVAL, "bad precision");
  if (!c->have_gauge) return fail(c, SSCG_ESTATE, "no gauge field set");
  HIPCHK(c, hipSetDevice(c->device));
  const size_t es = prec == SSCG_FP64 ? sizeof(double2) : sizeof(float2);
  CHK(ensure(c, c->apply_in, (size_t)nsrc * c->n * es));
  CHK(ensure(c, c->apply_out, (size_t)nsrc * c->n * es));
  return sscg::apply_A_staged(c, x, y, nsrc, prec, c->apply_in.p, c->apply_out.p, true);
}

}  // extern "C"

// y = A x through the planar staging buffers stage_in / stage_out (each nsrc * n
// complex numbers of the precision): pack, dslash, unpack on the caller's stream.
// tune = false never times launch shapes (no events, no host waits): the shape tuned
// earlier for (prec, nsrc) is used if there is one, else the context's default.
int sscg::apply_A_staged(sscg_ctx *c, const void *x, void *y, int nsrc, int prec, void *stage_in, void *stage_out,
                         bool tune) {
  hipStream_t st = c->user;
  launch_pack(x, stage_in, prec, nsrc, c->V, st);
  auto shape = [&]() -> Tune {
    if (tune) return apply_tune(c, stage_in, stage_out, nsrc, prec, st);
    auto it = c->tuned.find("apply|" + std::to_string(prec) + "|" + std::to_string(nsrc));
    return it != c->tuned.end() ? it->second : c->tune;
  };
  if (c->profiling && tune) {
    // time the dslash alone (blocking) and add it to the dslash stage
    while (c->events.size() < 2) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
    const Tune t = shape();
    HIPCHK(c, hipEventRecord(c->events[0], st));
    dslash_with(c, t, stage_in, stage_out, nsrc, prec, 0, 0.0, nullptr, nullptr, st);
    HIPCHK(c, hipEventRecord(c->events[1], st));
    HIPCHK(c, hipEventSynchronize(c->events[1]));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->events[0], c->events[1]));
    c->stage_ms[ST_DSLASH] += ms;
    c->stage_calls[ST_DSLASH] += 1;
  } else {
    dslash_with(c, shape(), stage_in, stage_out, nsrc, prec, 0, 0.0, nullptr, nullptr, st);
  }
  launch_unpack(stage_out, prec, y, nsrc, c->V, st);
  HIPCHK(c, hipGetLastError());
  return SSCG_OK;
}

int sscg::context_check_apply(sscg_ctx *c, const void *x, const void *y, int nsrc, int prec, size_t *bytes_each) {
  if (!c || !x || !y || nsrc <= 0) return fail(c, SSCG_EINVAL, "bad argument");
  if (prec != SSCG_FP64 && prec != SSCG_MIXED) return fail(c, SSCG_EINVAL, "bad precision");
  if (!c->have_gauge) return fail(c, SSCG_ESTATE, "no gauge field set");
  *bytes_each = (size_t)nsrc * c->n * (prec == SSCG_FP64 ? sizeof(double2) : sizeof(float2));
  return SSCG_OK;
}
int sscg::context_device(const sscg_ctx *c) { return c->device; }
int sscg::context_fail(sscg_ctx *c, int code, const char *msg) { return fail(c, code, msg); }

extern "C" {

static int check_solve_args(sscg_ctx *c, const void *v, int nsrc, const double *z, int nshift,
                            const sscg_solve_opts *o, const void *y) {
  if (!c) return fail(nullptr, SSCG_EINVAL, "null context");
  if (!v || !z || !y || !o) return fail(c, SSCG_EINVAL, "null argument");
  if (nsrc <= 0 || nshift <= 0) return fail(c, SSCG_EINVAL, "nsrc and nshift must be positive");
  if (nshift > 4096) return fail(c, SSCG_EINVAL, "at most 4096 shifts");
  if (!(o->tol > 0) || o->maxiter <= 0) return fail(c, SSCG_EINVAL, "tol must be > 0 and maxiter > 0");
  if (o->prec != SSCG_FP64 && o->prec != SSCG_MIXED && o->prec != SSCG_MIXED_SHIFTS)
    return fail(c, SSCG_EINVAL, "bad precision");
  for (int j = 0; j < 2 * nshift; ++j)
    if (!std::isfinite(z[j])) return fail(c, SSCG_EINVAL, "non-finite shift");
  return SSCG_OK;
}

int sscg_shifted_cg_solve(sscg_ctx *c, const void *v, int32_t nsrc, const double *z, int32_t nshift,
                          double sigma_seed, const sscg_solve_opts *opts, void *y, int32_t *conv_iter,
                          double *true_res, int32_t *iters) {
  CHK(check_solve_args(c, v, nsrc, z, nshift, opts, y));
  if (!std::isfinite(sigma_seed)) return fail(c, SSCG_EINVAL, "non-finite seed shift");
  std::vector<Prob> P(1);
  P[0].c = c;
  P[0].v = v;
  P[0].L = nsrc;
  P[0].N = nshift;
  P[0].sigma = sigma_seed;
  P[0].z.assign(z, z + 2 * nshift);
  P[0].y = y;
  P[0].conv_iter = conv_iter;
  P[0].true_res = true_res;
  P[0].iters = iters;
  int rc = run_solve(P, *opts);
  if (rc == SSCG_ENOTCONV) c->err = "maxiter reached before every shift converged";
  if (rc == SSCG_EBREAKDOWN) c->err = "CG breakdown: <p, (sigma I - A) p> vanished or a scalar is not finite";
  if (rc == SSCG_EINACCURATE) c->err = "a shift's FP64 true residual exceeds true_factor * tol after the mixed solve";
  return rc;
}

int sscg_batch_solve(sscg_ctx *const *ctxs, int32_t nprob, const void *const *v, const int32_t *nsrc,
                     const double *const *z, const int32_t *nshift, const double *sigma_seed,
                     const sscg_solve_opts *opts, void *const *y, int32_t *const *conv_iter,
                     double *const *true_res, int32_t *const *iters) {
  if (!ctxs || nprob <= 0 || nprob > kMaxJobs || !v || !nsrc || !z || !nshift || !sigma_seed || !opts || !y)
    return fail(ctxs ? ctxs[0] : nullptr, SSCG_EINVAL, "bad batch arguments (1..8 problems)");
  std::vector<Prob> P(nprob);
  for (int i = 0; i < nprob; ++i) {
    CHK(check_solve_args(ctxs[i], v[i], nsrc[i], z[i], nshift[i], opts, y[i]));
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return fail(ctxs[i], SSCG_EINVAL, "a context appears twice in a batch");
    P[i].c = ctxs[i];
    P[i].v = v[i];
    P[i].L = nsrc[i];
    P[i].N = nshift[i];
    P[i].sigma = sigma_seed[i];
    P[i].z.assign(z[i], z[i] + 2 * nshift[i]);
    P[i].y = y[i];
    P[i].conv_iter = conv_iter ? conv_iter[i] : nullptr;
    P[i].true_res = true_res ? true_res[i] : nullptr;
    P[i].iters = iters ? iters[i] : nullptr;
  }
  return run_solve(P, *opts);
}

int sscg_ss_moments(sscg_ctx *c, const void *y, int32_t nsrc, int32_t nshift, const double *cf, int32_t nmom,
                    void *s) {
  if (!c || !y || !cf || !s || nsrc <= 0 || nshift <= 0 || nmom <= 0) return fail(c, SSCG_EINVAL, "bad argument");
  if (nshift > 512) return fail(c, SSCG_EINVAL, "at most 512 shifts per moment sum");
  HIPCHK(c, hipSetDevice(c->device));
  CHK(ensure(c, c->small, (size_t)nmom * nshift * 2 * sizeof(double)));
  hipStream_t st = c->user;
  HIPCHK(c, hipMemcpyAsync(c->small.p, cf, (size_t)nmom * nshift * 2 * sizeof(double), hipMemcpyHostToDevice, st));
  launch_moments(y, nsrc, nshift, (const double *)c->small.p, nmom, s, c->n, st);
  // the coefficient buffer must outlive the kernel: order later host writes after it
  HIPCHK(c, hipStreamSynchronize(st));
  return SSCG_OK;
}

void sscg_default_ss_params(sscg_ss_params *p) {
  if (!p) return;
  p->gamma = 0.0;
  p->rho = 0.1;
  p->beta = 0.25;
  p->N = 32;
  p->M = 16;
  p->Nprime = 0;
  p->path = SSCG_PATH_LINES;
  p->method = SSCG_RR;
  p->rank_tol = 1e-7;
  p->spur_tol = 1e-6;
  p->npairs = 1;
  p->moments_in_loop = 0;
  p->weighted_tol = 0;
  p->seed_mode = 0;
  sscg_default_opts(&p->solve);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// extraction (Sec. 2.1): Rayleigh-Ritz or block Hankel, then acceptance (Sec. 3)

// C (na x nb, row-major on host, complex) = A^H B over n rows; A, B device column sets.
// herm: the product is Hermitian (A^H A, or Q^H (A Q) with A Hermitian; na = nb): the
// device computes the tiles on and above the diagonal, and the entries below the
// diagonal are the conjugates of those above.
static int gram(sscg_ctx *c, const void *A, int na, const void *B, int nb, std::vector<cd> &out, hipStream_t st,
                bool herm = false) {
  if (herm && na != nb) return fail(c, SSCG_EINVAL, "internal: Hermitian product of unequal sizes");
  // row chunks: enough blocks to spread over the chip, at least 64 rows each (more
  // chunks also mean more partials to sum afterwards)
  const int tiles = gemm_cn_tiles(na, nb, herm ? 1 : 0);
  // three 256-thread blocks fit per CU: about three per CU in all
  int nchunk = std::max(1, std::min(256, 768 / tiles));
  nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(nchunk, c->n / 64));
  const size_t nout = (size_t)na * nb;
  CHK(ensure(c, c->small, nchunk * nout * 2 * sizeof(double) + nout * 2 * sizeof(double)));
  double *part = (double *)c->small.p;
  double *red = part + nchunk * nout * 2;
  launch_gemm_cn(A, c->n, na, B, c->n, nb, c->n, part, nchunk, herm ? 1 : 0, st);
  launch_reduce_partials(part, nchunk, (int)(2 * nout), red, st);
  std::vector<double> h(2 * nout);
  HIPCHK(c, hipMemcpyAsync(h.data(), red, 2 * nout * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  out.resize(nout);
  for (size_t k = 0; k < nout; ++k) out[k] = cd(h[2 * k], h[2 * k + 1]);
  if (herm)
    for (int a = 1; a < na; ++a)
      for (int b = 0; b < a; ++b) out[(size_t)a * nb + b] = std::conj(out[(size_t)b * nb + a]);
  return SSCG_OK;
}

// C = A T (and C2 = A2 T when A2 is given) with T (na x nb) row-major host complex;
// upper: T is upper triangular (the products skip its zero part). Stream-ordered: T
// goes through the context's host staging vector, which the next call only rewrites
// after a synchronisation (every caller reads a Gram matrix or residuals back between
// two calls).
static int basis_change(sscg_ctx *c, const void *A, int na, const std::vector<cd> &T, int nb, void *C,
                        hipStream_t st, const void *A2 = nullptr, void *C2 = nullptr, bool upper = false) {
  const size_t need = (size_t)na * nb * sizeof(double2);
  if (c->tmp.bytes < need) {  // a kernel still reading the old buffer finishes first
    HIPCHK(c, hipStreamSynchronize(st));
    CHK(ensure(c, c->tmp, need));
  }
  std::vector<double> &h = c->hstage;
  h.resize(2 * (size_t)na * nb);
  for (size_t k = 0; k < (size_t)na * nb; ++k) {
    h[2 * k] = T[k].real();
    h[2 * k + 1] = T[k].imag();
  }
  HIPCHK(c, hipMemcpyAsync(c->tmp.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
  launch_gemm_nn(A, c->n, na, (const double *)c->tmp.p, nb, C, c->n, c->n, upper ? 1 : 0, st);
  if (A2) launch_gemm_nn(A2, c->n, na, (const double *)c->tmp.p, nb, C2, c->n, c->n, upper ? 1 : 0, st);
  return SSCG_OK;
}

// Hermitian eigen-decomposition of a row-major n x n complex matrix (uses the
// column-major routine on the transpose; for a Hermitian matrix the transpose is
// the conjugate, whose eigenvectors are the conjugates).
static bool eig_rowmajor(int n, const std::vector<cd> &A, std::vector<double> &ev, std::vector<cd> &W) {
  std::vector<double> a(2 * (size_t)n * n), vv(2 * (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {  // column-major element (i, j) = A[i][j]
      a[2 * (i + (size_t)n * j)] = A[(size_t)i * n + j].real();
      a[2 * (i + (size_t)n * j) + 1] = A[(size_t)i * n + j].imag();
    }
  ev.resize(n);
  const bool ok = herm_eig(n, a.data(), ev.data(), vv.data());
  W.resize((size_t)n * n);  // row-major: W[i][k] = component i of eigenvector k
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) W[(size_t)i * n + k] = cd(vv[2 * (i + (size_t)n * k)], vv[2 * (i + (size_t)n * k) + 1]);
  return ok;
}
#define EIGCHK(ctx, call) \
  do { \
    if (!(call)) return fail(ctx, SSCG_ENOTCONV, "dense Hermitian eigensolver did not converge"); \
  } while (0)

static int apply_A_planar(sscg_ctx *c, const void *X, void *AX, int ncol, hipStream_t st) {
  const size_t vec = c->n * sizeof(double2);
  for (int k = 0; k < ncol; k += 8) {
    const int cnt = std::min(8, ncol - k);
    const void *xin = (const char *)X + k * vec;
    void *xout = (char *)AX + k * vec;
    dslash_with(c, apply_tune(c, xin, xout, cnt, 0, st), xin, xout, cnt, 0, 0, 0.0, nullptr, nullptr, st);
  }
  return SSCG_OK;
}

// residual norms ||AX_c - lam_c X_c|| and ||X_c||
static int col_residuals(sscg_ctx *c, const void *AX, const void *X, int ncol, const std::vector<double> &lam,
                         std::vector<double> &res, std::vector<double> &xn, hipStream_t st) {
  const int nchunk = 64;
  CHK(ensure(c, c->small, (size_t)(2 * ncol * nchunk + ncol) * sizeof(double)));
  double *part = (double *)c->small.p;
  double *ldev = part + 2 * ncol * nchunk;
  HIPCHK(c, hipMemcpyAsync(ldev, lam.data(), ncol * sizeof(double), hipMemcpyHostToDevice, st));
  launch_resid_cols(AX, X, c->n, ncol, ldev, c->n, part, nchunk, st);
  std::vector<double> h((size_t)2 * ncol * nchunk);
  HIPCHK(c, hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  res.assign(ncol, 0.0);
  xn.assign(ncol, 0.0);
  for (int k = 0; k < ncol; ++k)
    for (int b = 0; b < nchunk; ++b) {
      res[k] += h[(size_t)k * nchunk + b];
      xn[k] += h[(size_t)(ncol + k) * nchunk + b];
    }
  for (int k = 0; k < ncol; ++k) {
    xn[k] = std::sqrt(xn[k]);
    res[k] = std::sqrt(res[k]) / (xn[k] > 0 ? xn[k] : 1.0);
  }
  return SSCG_OK;
}

// Rayleigh-Ritz on the columns of S (n x ncol): Q from two Gram passes over the
// unit-norm columns (the second restores the orthogonality the first loses),
// keeping directions whose singular value exceeds rank_tol times the largest; then
// A~ = Q^H (A Q), its eigenpairs, X = Q W and A X = (A Q) W in Xd / AXd.
// Only the Ritz values that the caller's filter `want` keeps get their vectors: X
// and A X hold them in order, and `sel` lists their indices into lam (the acceptance
// rectangle discards the others, so their vectors are never needed).
template <typename Want>
static int extract_rr(sscg_ctx *c, const void *S, int ncol, double rank_tol, void *Xd, void *AXd,
                      std::vector<double> &lam, int &r, std::vector<int> &sel, Want &&want, hipStream_t st) {
  const size_t vec = c->n * sizeof(double2);
  std::vector<cd> G;
  CHK(gram(c, S, ncol, S, ncol, G, st, true));
  std::vector<double> dsc(ncol);
  for (int a = 0; a < ncol; ++a) dsc[a] = G[(size_t)a * ncol + a].real() > 0 ? 1.0 / std::sqrt(G[(size_t)a * ncol + a].real()) : 0.0;
  std::vector<cd> Gs((size_t)ncol * ncol);
  for (int a = 0; a < ncol; ++a)
    for (int b = 0; b < ncol; ++b) Gs[(size_t)a * ncol + b] = dsc[a] * G[(size_t)a * ncol + b] * dsc[b];
  std::vector<double> ev;
  std::vector<cd> W;
  EIGCHK(c, eig_rowmajor(ncol, Gs, ev, W));
  const double emax = ev.back();
  std::vector<int> keep;
  for (int k = ncol - 1; k >= 0; --k)
    if (emax > 0 && ev[k] > rank_tol * rank_tol * emax) keep.push_back(k);
  r = (int)keep.size();
  lam.clear();
  if (r == 0) return SSCG_OK;
  std::vector<cd> T1((size_t)ncol * r);
  for (int a = 0; a < ncol; ++a)
    for (int q = 0; q < r; ++q) T1[(size_t)a * r + q] = dsc[a] * W[(size_t)a * ncol + keep[q]] / std::sqrt(ev[keep[q]]);
  CHK(ensure(c, c->Qbuf, (size_t)r * vec));
  CHK(ensure(c, c->AQbuf, (size_t)r * vec));
  CHK(basis_change(c, S, ncol, T1, r, c->AQbuf.p, st));  // Q1 (held in AQbuf for now)
  std::vector<cd> G2;
  CHK(gram(c, c->AQbuf.p, r, c->AQbuf.p, r, G2, st, true));
  // second pass: Q1 is orthonormal up to rounding, so its Gram matrix is close to I and
  // a Cholesky factor G2 = R^H R gives Q = Q1 R^-1 (an eigen-decomposition of G2 is
  // the fallback if a pivot is not positive)
  std::vector<cd> T2;
  const bool chol = chol_inverse_upper(r, G2, T2);  // T2 = R^-1, upper triangular
  if (!chol) {
    std::vector<double> ev2;
    std::vector<cd> W2;
    EIGCHK(c, eig_rowmajor(r, G2, ev2, W2));
    T2.assign((size_t)r * r, cd(0, 0));
    for (int a = 0; a < r; ++a)
      for (int q = 0; q < r; ++q) T2[(size_t)a * r + q] = W2[(size_t)a * r + q] / std::sqrt(std::max(ev2[q], 1e-300));
  }
  CHK(basis_change(c, c->AQbuf.p, r, T2, r, c->Qbuf.p, st, nullptr, nullptr, chol));  // Q
  CHK(apply_A_planar(c, c->Qbuf.p, c->AQbuf.p, r, st));         // A Q
  std::vector<cd> At;
  CHK(gram(c, c->Qbuf.p, r, c->AQbuf.p, r, At, st, true));  // Hermitian since A is
  std::vector<cd> Wr;
  EIGCHK(c, eig_rowmajor(r, At, lam, Wr));
  sel.clear();
  for (int k = 0; k < r; ++k)
    if (want(lam[k])) sel.push_back(k);
  const int m = (int)sel.size();
  if (m == 0) return SSCG_OK;
  std::vector<cd> Wsel((size_t)r * m);
  for (int a = 0; a < r; ++a)
    for (int i = 0; i < m; ++i) Wsel[(size_t)a * m + i] = Wr[(size_t)a * r + sel[i]];
  CHK(basis_change(c, c->Qbuf.p, r, Wsel, m, Xd, st, c->AQbuf.p, AXd));
  (void)vec;
  return SSCG_OK;
}

// Block Hankel on moments mu_k = V^H s_k (k < 2M) built from Gv[a][l N_all + off + j]
// = <v_a, y_{l, off + j}>: H = [M_{i+j}], H< = [M_{i+j+1}] (L x L blocks). H is
// Hermitian positive semidefinite for the real filters used here, so the pencil is
// reduced on H's dominant eigenvectors and solved as a Hermitian problem; the
// eigenvectors are X = S_hat u (S_hat = first M moments, columns k L + l).
// Block moments mu_k = V^H s_k (k < 2M, L x L blocks, [k][a][l]) from the Gram
// entries <v_a, y_{l,j}> of the stored solutions of one pair (nodes off .. off+N-1).
static std::vector<cd> block_moments_from_solutions(const std::vector<cd> &Gv, int L, int Nall, int off, int N,
                                                    int M, const std::vector<cd> &zeta, const std::vector<cd> &w) {
  const int K = 2 * M;
  std::vector<cd> mu((size_t)K * L * L, cd(0, 0));
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < N; ++j) {
      const cd cc = w[j] * std::pow(zeta[j], k);
      for (int a = 0; a < L; ++a)
        for (int l = 0; l < L; ++l) mu[((size_t)k * L + a) * L + l] += cc * Gv[(size_t)a * L * Nall + (size_t)l * Nall + off + j];
    }
  return mu;
}

// Block Hankel extraction from the block moments mu ([2M][L][L]) and the moment
// vectors S (columns k L + l, k < M).
static int extract_hankel(sscg_ctx *c, const std::vector<cd> &mu, int L, int M, double gamma, double rho,
                          double rank_tol, const void *S, void *Xd, void *AXd, std::vector<double> &lam, int &r,
                          hipStream_t st) {
  const int m = M * L;
  std::vector<cd> H((size_t)m * m), Hs((size_t)m * m);
  for (int bi = 0; bi < M; ++bi)
    for (int bj = 0; bj < M; ++bj)
      for (int a = 0; a < L; ++a)
        for (int l = 0; l < L; ++l) {
          H[(size_t)(bi * L + a) * m + bj * L + l] = mu[((size_t)(bi + bj) * L + a) * L + l];
          Hs[(size_t)(bi * L + a) * m + bj * L + l] = mu[((size_t)(bi + bj + 1) * L + a) * L + l];
        }
  std::vector<double> ev;
  std::vector<cd> W;
  EIGCHK(c, eig_rowmajor(m, H, ev, W));
  const double emax = ev.back();
  std::vector<int> keep;
  for (int k = m - 1; k >= 0; --k)
    if (emax > 0 && ev[k] > rank_tol * emax) keep.push_back(k);
  r = (int)keep.size();
  lam.clear();
  if (r == 0) return SSCG_OK;
  std::vector<cd> Wr((size_t)m * r);
  for (int a = 0; a < m; ++a)
    for (int q = 0; q < r; ++q) Wr[(size_t)a * r + q] = W[(size_t)a * m + keep[q]] / std::sqrt(ev[keep[q]]);
  std::vector<cd> red((size_t)r * r, cd(0, 0));
  for (int q1 = 0; q1 < r; ++q1)
    for (int q2 = 0; q2 < r; ++q2) {
      cd acc = 0;
      for (int a = 0; a < m; ++a) {
        cd t = 0;
        for (int b = 0; b < m; ++b) t += Hs[(size_t)a * m + b] * Wr[(size_t)b * r + q2];
        acc += std::conj(Wr[(size_t)a * r + q1]) * t;
      }
      red[(size_t)q1 * r + q2] = acc;
    }
  std::vector<double> eta;
  std::vector<cd> T;
  EIGCHK(c, eig_rowmajor(r, red, eta, T));
  lam.resize(r);
  for (int q = 0; q < r; ++q) lam[q] = gamma + rho * eta[q];
  std::vector<cd> Tc((size_t)m * r, cd(0, 0));
  for (int a = 0; a < m; ++a)
    for (int q = 0; q < r; ++q) {
      cd acc = 0;
      for (int b = 0; b < r; ++b) acc += Wr[(size_t)a * r + b] * T[(size_t)b * r + q];
      Tc[(size_t)a * r + q] = acc;
    }
  CHK(basis_change(c, S, m, Tc, r, Xd, st));
  CHK(apply_A_planar(c, Xd, AXd, r, st));
  return SSCG_OK;
}

extern "C" int sscg_ss_eigs(sscg_ctx *c, const sscg_ss_params *p, const void *v, int32_t nsrc, int32_t max_eigs,
                            double *lambda, void *X, double *res, int32_t *n_found, sscg_ss_info *info) {
  if (!c || !p || !v || nsrc <= 0 || max_eigs < 0 || (max_eigs > 0 && (!lambda || !res)) || !n_found)
    return fail(c, SSCG_EINVAL, "bad argument");
  const int P = p->npairs > 1 ? p->npairs : 1;
  if (p->M <= 0 || p->N < 4 || (p->path == SSCG_PATH_LINES && p->N % 2) || !(p->rho > 0) ||
      (p->path == SSCG_PATH_LINES && !(p->beta > 0)) || (p->path != SSCG_PATH_LINES && p->path != SSCG_PATH_CIRCLE))
    return fail(c, SSCG_EINVAL, "bad contour parameters");
  if (p->method != SSCG_RR && p->method != SSCG_HANKEL) return fail(c, SSCG_EINVAL, "bad extraction method");
  if (p->method == SSCG_HANKEL && 2 * p->M > p->N)
    return fail(c, SSCG_EINVAL, "Hankel needs 2M <= N moments from N nodes");
  if (!(p->rank_tol > 0 && p->rank_tol < 1)) return fail(c, SSCG_EINVAL, "rank_tol must lie in (0, 1)");
  if (p->seed_mode < 0 || p->seed_mode > 2) return fail(c, SSCG_EINVAL, "seed_mode must be 0, 1 or 2");
  if (p->N > 512 || (int64_t)p->M * nsrc > 256)
    return fail(c, SSCG_EINVAL, "at most 512 nodes and M * nsrc <= 256 moment columns");
  const int Np = p->Nprime ? p->Nprime : p->N;
  if (p->path == SSCG_PATH_LINES && (Np < 4 || Np % 2 || Np > p->N)) return fail(c, SSCG_EINVAL, "bad Nprime");
  if (P > 1 && p->path != SSCG_PATH_LINES) return fail(c, SSCG_EINVAL, "adjacent pairs need the line path");
  if (P > 64) return fail(c, SSCG_EINVAL, "at most 64 adjacent pairs");
  HIPCHK(c, hipSetDevice(c->device));
  const int N = p->N, M = p->M, L = nsrc;
  const size_t n = c->n, vec = n * sizeof(double2);
  // normalised nodes and weights of one pair (identical for every pair)
  std::vector<cd> zt, zeta, w;
  if (p->path == SSCG_PATH_LINES) quad_lines_host(N, 0.0, 1.0, p->beta, zt, zeta, w);
  else quad_circle_host(N, 0.0, 1.0, zt, zeta, w);
  // distinct nodes of all pairs (Sec. 3: neighbouring pairs share all but N' - 2 nodes)
  std::vector<cd> z_all;
  std::vector<int> offsets(P);
  std::vector<double> centres(P);
  if (P == 1) {
    for (int j = 0; j < N; ++j) z_all.push_back(p->gamma + p->rho * zeta[j]);
    offsets[0] = 0;
    centres[0] = p->gamma;
  } else {
    const double h = 2.0 * p->rho / (N / 2 - 1);
    const int step = (Np - 2) / 2;
    const int total_x = N / 2 + (P - 1) * step;
    const double span = (P - 1) * step * h;
    for (int i = 0; i < total_x; ++i) {
      const double x = (p->gamma - 0.5 * span - p->rho) + h * i;
      z_all.push_back(cd(x, p->beta * p->rho));
      z_all.push_back(cd(x, -p->beta * p->rho));
    }
    for (int q = 0; q < P; ++q) {
      offsets[q] = 2 * step * q;
      centres[q] = p->gamma - 0.5 * span + step * h * q;
    }
  }
  const int Nall = (int)z_all.size();
  if (Nall > 4096) return fail(c, SSCG_EINVAL, "too many distinct nodes");
  const bool in_loop = p->moments_in_loop != 0;
  // moments per pair: M for Rayleigh-Ritz; 2M for Hankel when they are summed in the
  // loop (its block moments V^H s_k run to k = 2M - 1)
  const int K = (in_loop && p->method == SSCG_HANKEL) ? 2 * M : M;
  if (in_loop && (P * K > 32 || p->solve.prec == SSCG_MIXED))
    return fail(c, SSCG_EINVAL, "in-loop moments need npairs * M (2M for Hankel) <= 32 and an FP64 seed");
  // the in-loop update addresses a moment vector with 32-bit byte offsets
  if (in_loop && (int64_t)c->n * 16 >= ((int64_t)1 << 31))
    return fail(c, SSCG_EINVAL, "in-loop moments need 12 V < 134217728 (vectors under 2 GiB)");
  const int ncol = M * L;
  // moment coefficients c[k][j] = w_j zeta_j^k of one pair (eq. 2), k < K
  std::vector<double> cf(2 * (size_t)K * N);
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < N; ++j) {
      const cd cc = w[j] * std::pow(zeta[j], k);
      cf[2 * ((size_t)k * N + j)] = cc.real();
      cf[2 * ((size_t)k * N + j) + 1] = cc.imag();
    }
  hipStream_t st = c->work;
  // largest moment coefficient per distinct node over every pair it belongs to
  std::vector<double> cmax(Nall, 0.0);
  for (int q = 0; q < P; ++q)
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < N; ++j)
        cmax[offsets[q] + j] = std::max(cmax[offsets[q] + j], std::hypot(cf[2 * ((size_t)k * N + j)],
                                                                           cf[2 * ((size_t)k * N + j) + 1]));
  if (in_loop) {
    // pair q's moments are rows q K .. q K + K - 1 of one [P K][Nall] coefficient
    // matrix over the distinct nodes (zero outside the pair's N nodes), so the
    // moment sums of every pair are accumulated by the one solve
    std::vector<double> cm(2 * (size_t)P * K * Nall, 0.0);
    for (int q = 0; q < P; ++q)
      for (int k = 0; k < K; ++k)
        for (int j = 0; j < N; ++j) {
          const size_t dst = 2 * ((size_t)(q * K + k) * Nall + offsets[q] + j);
          cm[dst] = cf[2 * ((size_t)k * N + j)];
          cm[dst + 1] = cf[2 * ((size_t)k * N + j) + 1];
        }
    CHK(ensure(c, c->cmom, cm.size() * sizeof(double)));
    CHK(ensure(c, c->Sbuf, (size_t)P * K * L * vec));
    HIPCHK(c, hipMemcpyAsync(c->cmom.p, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemsetAsync(c->Sbuf.p, 0, (size_t)P * K * L * vec, st));
  } else {
    // one shifted CG for all distinct nodes into the internal (planar) solution buffer
    CHK(ensure(c, c->Ybuf, (size_t)L * Nall * vec));
  }
  std::vector<double> zd(2 * Nall);
  for (int j = 0; j < Nall; ++j) {
    zd[2 * j] = z_all[j].real();
    zd[2 * j + 1] = z_all[j].imag();
  }
  std::vector<Prob> PP(1);
  PP[0].c = c;
  PP[0].v = v;
  PP[0].L = L;
  PP[0].N = Nall;
  // seed shift: the interval centre, or a shift outside the spectrum (|A| <= 1 + 8
  // kappa for r = 1) where sigma I - A is positive definite
  const int seed_mode = p->seed_mode != 0 ? p->seed_mode : 1;
  PP[0].sigma = seed_mode == 2 ? 1.0 + 8.0 * std::fabs(c->kappa) + 0.25 : p->gamma;
  PP[0].z = zd;
  PP[0].y = in_loop ? nullptr : c->Ybuf.p;
  PP[0].keep_planar = true;
  if (p->weighted_tol) {
    const double m = *std::max_element(cmax.begin(), cmax.end());
    PP[0].tscale.resize(Nall);
    for (int j = 0; j < Nall; ++j) PP[0].tscale[j] = cmax[j] > m * 1e-12 ? m / cmax[j] : 1e12;
  }
  if (in_loop) {
    PP[0].mom = c->Sbuf.p;
    PP[0].mom_coef = c->cmom.p;
    PP[0].nmom = P * K;
  }
  std::vector<int32_t> iters(L), conv((size_t)L * Nall);
  PP[0].iters = iters.data();
  PP[0].conv_iter = conv.data();
  auto t0 = std::chrono::steady_clock::now();
  int rc = run_solve(PP, p->solve);
  if (rc != SSCG_OK && rc != SSCG_ENOTCONV && rc != SSCG_EINACCURATE) return rc;
  auto t1 = std::chrono::steady_clock::now();
  double t_mom = 0.0;
  if (!in_loop) CHK(ensure(c, c->Sbuf, (size_t)ncol * vec));
  // X and AX buffers live in the shift workspace (free after the solve) when large enough
  void *Xd = nullptr, *AXd = nullptr;
  if (c->W.bytes >= 2 * (size_t)ncol * vec) {
    Xd = c->W.p;
    AXd = (char *)c->W.p + (size_t)ncol * vec;
  } else {
    CHK(ensure(c, c->Xbuf, (size_t)ncol * vec));
    CHK(ensure(c, c->AXbuf, (size_t)ncol * vec));
    Xd = c->Xbuf.p;
    AXd = c->AXbuf.p;
  }
  std::vector<cd> Gv;
  if (p->method == SSCG_HANKEL && !in_loop) {
    CHK(ensure(c, c->v64, (size_t)L * vec));
    launch_pack(v, c->v64.p, 0, L, c->V, st);
    CHK(gram(c, c->v64.p, L, c->Ybuf.p, L * Nall, Gv, st));  // [a][l Nall + j] = <v_a, y_{l,j}>
  }
  // accepted pairs kept: at most max_eigs nearest gamma, their vectors in Acc slots
  struct Acc {
    double lam, res, dist;
    int slot;
  };
  std::vector<Acc> acc;
  int total_found = 0, rank_max = 0, ncand = 0;
  int64_t ext_bytes = 0;
  if (X && max_eigs > 0) CHK(ensure(c, c->Accbuf, (size_t)max_eigs * vec));
  for (int q = 0; q < P; ++q) {
    const void *Sq = c->Sbuf.p;
    if (in_loop) {
      Sq = (const char *)c->Sbuf.p + (size_t)q * K * L * vec;
    } else {
      auto tm0 = std::chrono::steady_clock::now();
      CHK(ensure(c, c->small, cf.size() * sizeof(double)));
      HIPCHK(c, hipMemcpyAsync(c->small.p, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice, st));
      launch_moments_strided2((const char *)c->Ybuf.p + (size_t)offsets[q] * vec, L, N, (int64_t)Nall,
                              (const double *)c->small.p, M, c->Sbuf.p, (int64_t)n, 1, L, st);
      HIPCHK(c, hipStreamSynchronize(st));
      t_mom += std::chrono::duration<double>(std::chrono::steady_clock::now() - tm0).count();
    }
    // acceptance (Sec. 3): the rectangle of the N' nodes nearest this pair's centre;
    // half-open on the right except for the last pair, so a shared edge counts once
    double lo, hi;
    if (p->path == SSCG_PATH_LINES) {
      std::vector<double> xr;
      for (int j = 0; j < N; j += 2) xr.push_back(zeta[j].real());
      std::vector<int> ord(xr.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::fabs(xr[a]) < std::fabs(xr[b]); });
      double mn = 1e300, mx = -1e300;
      for (int i = 0; i < Np / 2; ++i) {
        mn = std::min(mn, xr[ord[i]]);
        mx = std::max(mx, xr[ord[i]]);
      }
      lo = centres[q] + p->rho * mn;
      hi = centres[q] + p->rho * mx;
    } else {
      lo = centres[q] - p->rho;
      hi = centres[q] + p->rho;
    }
    auto inside = [&](double x) { return x >= lo && (q < P - 1 ? x < hi : x <= hi); };
    std::vector<double> lam;
    std::vector<int> sel;  // candidates whose vectors are in Xd / AXd, in order
    int r = 0;
    if (p->method == SSCG_RR) {
      CHK(extract_rr(c, Sq, ncol, p->rank_tol, Xd, AXd, lam, r, sel, inside, st));
    } else {
      std::vector<cd> mu;
      if (in_loop) {
        // mu_k = V^H s_k from the 2M moment vectors summed in the loop
        std::vector<cd> Gs;
        CHK(gram(c, c->v64.p, L, Sq, K * L, Gs, st));  // [a][k L + l]
        mu.assign((size_t)K * L * L, cd(0, 0));
        for (int k = 0; k < K; ++k)
          for (int a = 0; a < L; ++a)
            for (int l = 0; l < L; ++l) mu[((size_t)k * L + a) * L + l] = Gs[(size_t)a * K * L + (size_t)k * L + l];
      } else {
        mu = block_moments_from_solutions(Gv, L, Nall, offsets[q], N, M, zeta, w);
      }
      CHK(extract_hankel(c, mu, L, M, centres[q], p->rho, p->rank_tol, Sq, Xd, AXd, lam, r, st));
      sel.resize(r);
      for (int k = 0; k < r; ++k) sel[k] = k;
    }
    rank_max = std::max(rank_max, r);
    ncand += r;
    // device memory of this pair's extraction: the moment vectors S (n x M L); for
    // Rayleigh-Ritz the basis Q and A Q (r vectors each); the vectors X and A X of the
    // candidates (the r Hankel ones, the Ritz ones inside the rectangle; the buffers
    // are reused from pair to pair)
    const int nsel = (int)sel.size();
    ext_bytes = std::max(ext_bytes, (int64_t)((size_t)ncol + (p->method == SSCG_RR ? 2 * (size_t)r : 0) +
                                              2 * (size_t)nsel) * (int64_t)vec);
    if (nsel == 0) continue;
    std::vector<double> lsel(nsel), rs, xn;
    for (int i = 0; i < nsel; ++i) lsel[i] = lam[sel[i]];
    CHK(col_residuals(c, AXd, Xd, nsel, lsel, rs, xn, st));
    for (int i = 0; i < nsel; ++i) {
      const int k = sel[i];
      if (!inside(lam[k]) || !(rs[i] <= p->spur_tol)) continue;
      ++total_found;
      if (max_eigs == 0) continue;
      const double dist = std::fabs(lam[k] - p->gamma);
      int slot = -1;
      if ((int)acc.size() < max_eigs) {
        slot = (int)acc.size();
        acc.push_back({lam[k], rs[i], dist, slot});
      } else {
        auto worst = std::max_element(acc.begin(), acc.end(), [](const Acc &a, const Acc &b) { return a.dist < b.dist; });
        if (worst->dist <= dist) continue;
        slot = worst->slot;
        *worst = {lam[k], rs[i], dist, slot};
      }
      if (X) {
        // unit-normalised copy of the candidate's vector into its slot
        std::vector<double> one(1, xn[i] > 0 ? 1.0 / xn[i] : 1.0);
        char *dst = (char *)c->Accbuf.p + (size_t)slot * vec;
        HIPCHK(c, hipMemcpyAsync(dst, (const char *)Xd + (size_t)i * vec, vec, hipMemcpyDeviceToDevice, st));
        CHK(ensure(c, c->small, sizeof(double)));
        HIPCHK(c, hipMemcpyAsync(c->small.p, one.data(), sizeof(double), hipMemcpyHostToDevice, st));
        launch_colscale(dst, (int64_t)n, 1, (const double *)c->small.p, (int64_t)n, st);
        HIPCHK(c, hipStreamSynchronize(st));
      }
    }
  }
  std::sort(acc.begin(), acc.end(), [](const Acc &a, const Acc &b) { return a.lam < b.lam; });
  *n_found = total_found;
  for (size_t i = 0; i < acc.size(); ++i) {
    lambda[i] = acc[i].lam;
    res[i] = acc[i].res;
    if (X) launch_unpack((const char *)c->Accbuf.p + (size_t)acc[i].slot * vec, 0, (char *)X + i * vec, 1, c->V, st);
  }
  HIPCHK(c, hipStreamSynchronize(st));
  auto t3 = std::chrono::steady_clock::now();
  if (info) {
    info->rank = rank_max;
    info->n_candidates = ncand;
    info->iters = *std::max_element(iters.begin(), iters.end());
    info->solve_status = rc;
    info->t_solve = std::chrono::duration<double>(t1 - t0).count();
    info->t_moments = t_mom;
    info->t_extract = std::chrono::duration<double>(t3 - t1).count() - t_mom;
    int64_t su = 0, mv = 0;
    for (int l = 0; l < L; ++l) {
      mv += iters[l];
      for (int j = 0; j < Nall; ++j) {
        const int ci = conv[(size_t)l * Nall + j];
        su += ci >= 0 ? ci : iters[l];
      }
    }
    info->shift_updates = su;
    info->matvecs = mv + ncand;  // seed products plus A Q (Rayleigh-Ritz) or A X (Hankel)
    const int ks = PP[0].switch_iter;
    int64_t su32 = 0, it32 = 0;
    if (ks >= 0)
      for (int l = 0; l < L; ++l) {
        it32 += std::max(0, iters[l] - ks);
        for (int j = 0; j < Nall; ++j) {
          const int ci = conv[(size_t)l * Nall + j];
          su32 += std::max(0, (ci >= 0 ? ci : iters[l]) - ks);
        }
      }
    info->shift_updates_fp32 = su32;
    info->seed_iters = mv;
    info->seed_iters_fp32 = it32;
    info->switch_iter = ks;
    info->max_true_res = PP[0].max_true_res;
    info->extract_bytes = ext_bytes + (X && max_eigs > 0 ? (int64_t)max_eigs * (int64_t)vec : 0);
  }
  return rc == SSCG_ENOTCONV || rc == SSCG_EINACCURATE ? rc : SSCG_OK;
}
