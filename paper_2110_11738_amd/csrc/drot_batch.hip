// Host side of the batched solver: many independent OT problems of different
// shapes advance together, one batched sweep launch and one batched aux launch
// per iteration over work lists of (problem, work item) pairs.  Every problem
// keeps its own device state and stopping test (Algorithm 1 and the stopping
// criteria of Section 3, per problem); finished problems are dropped from the
// work lists when the lists are rebuilt.
//
// A sweep work item of problem b is one column strip of a group of row
// blocks (`rows` rows each, `blocks per item` of them, strided so that the
// items running at one moment stream neighbouring bands of rows).  The two
// numbers are chosen per size class of (m, n) -- a bucket of power-of-two
// ranges -- from the context's tuner cache, filled by drot_tune_batched,
// which times candidate schedules on the problems of each bucket.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/drot.h"
#include "drot_internal.h"

using namespace drot;

// Shared with drot_host.hip.
int drot_internal_fail(int code, const char* msg);
int drot_internal_ctx_prepare(drot_ctx* c, void** ws, size_t bytes);
double drot_internal_wall_rate(const drot_ctx* c);
bool drot_internal_batch_tile(const drot_ctx* c, int key, int* rows, int* per_item);
void drot_internal_set_batch_tile(drot_ctx* c, int key, int rows, int per_item);
int drot_internal_batch_chunks(const drot_ctx* c, int key);
void drot_internal_set_batch_chunks(drot_ctx* c, int key, int chunks);

namespace {

int bfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return drot_internal_fail(code, buf);
}

#define BHIP(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return bfail(DROT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr int kBatchTrace = 256;

struct ProbLayout {
  SweepGeom g;
  size_t off[12];
};

}  // namespace

namespace {

// Size class of a side: < 128, < 256, < 512, < 1024, < 2048, >= 2048.
int side_bucket(int64_t x) {
  int b = 0;
  while (b < 5 && x >= ((int64_t)128 << b)) ++b;
  return b;
}

// Key of the tuner cache: element type, cache policy and the two size classes.
int tile_key(int dtype, bool stream, int64_t m, int64_t n) {
  return ((dtype * 2 + (stream ? 1 : 0)) * 6 + side_bucket(m)) * 6 + side_bucket(n);
}

// Validation of a batch's arguments (before any device work).
int validate_batch(int32_t count, int dtype, const drot_problem* probs, const drot_params* prm) {
  if (count < 1) return bfail(DROT_EINVAL, "count must be >= 1");
  if (!probs || !prm) return bfail(DROT_EINVAL, "probs and params must be non-NULL");
  if (dtype != DROT_F32 && dtype != DROT_F64) return bfail(DROT_EINVAL, "unknown dtype %d", dtype);
  if (!(prm->max_iter >= 1)) return bfail(DROT_EINVAL, "max_iter must be >= 1");
  if (prm->tol_mode != DROT_TOL_RELATIVE && prm->tol_mode != DROT_TOL_ABSOLUTE)
    return bfail(DROT_EINVAL, "unknown tol_mode %d", prm->tol_mode);
  if (prm->flags & ~(DROT_FLAG_NO_GRAPH))
    return bfail(DROT_EUNSUPPORTED, "batched solves take only DROT_FLAG_NO_GRAPH");
  if (prm->tile_chunks < 0 || prm->tile_chunks > 2 || prm->tile_rows < 0 || prm->tile_rows > 4096 ||
      prm->tile_groups < 0)
    return bfail(DROT_EINVAL, "bad tile parameters");
  const size_t es = dtype == DROT_F32 ? 4 : 8;
  for (int b = 0; b < count; ++b) {
    const drot_problem& P = probs[b];
    if (P.m < 1 || P.n < 1 || P.ldc < P.n || P.ldx < P.n)
      return bfail(DROT_EINVAL, "problem %d: bad sizes or leading dimensions", b);
    if (!P.C || !P.p || !P.q || !P.X) return bfail(DROT_EINVAL, "problem %d: NULL array", b);
    if ((P.mu0 == nullptr) != (P.nu0 == nullptr))
      return bfail(DROT_EINVAL, "problem %d: mu0 and nu0 must be given together", b);
    if (!(P.rho > 0) || !std::isfinite(P.rho) || !(P.tol >= 0) || !std::isfinite(P.tol))
      return bfail(DROT_EINVAL, "problem %d: rho must be > 0 and tol >= 0", b);
    if ((uintptr_t)P.C % es || (uintptr_t)P.X % es || (uintptr_t)P.p % es || (uintptr_t)P.q % es)
      return bfail(DROT_EINVAL, "problem %d: arrays must be aligned to their element size", b);
    const uintptr_t c0 = (uintptr_t)P.C, c1 = c0 + (size_t)((P.m - 1) * P.ldc + P.n) * es;
    const uintptr_t x0 = (uintptr_t)P.X, x1 = x0 + (size_t)((P.m - 1) * P.ldx + P.n) * es;
    if (c0 < x1 && x0 < c1) return bfail(DROT_EINVAL, "problem %d: C and X overlap", b);
  }
  return DROT_OK;
}

// One batched run: layout, initialisation, iterations, final evaluation.
// Owns the pinned staging buffers, the capture stream and the graph; the
// device workspace is the context's.
struct BatchRun {
  drot_ctx* c = nullptr;
  int count = 0, dtype = 0;
  const drot_problem* probs = nullptr;
  drot_params prm{};
  TileCfg tile{1, 4, 4, false, false};
  std::vector<ProbLayout> L;
  size_t SS = 0, off_args = 0, off_sw = 0, off_aw = 0, total = 0;
  char* base = nullptr;
  SweepArgs* h_args = nullptr;
  uint2* h_sw = nullptr;
  uint2* h_aw = nullptr;
  char* h_st = nullptr;  // count records with stride SS
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t n_sw = 0, n_aw = 0, grid_sw = 0, max_sweep = 0, max_aux = 0;
  std::vector<char> active;
  double wall_rate = 1e8;

  DevState& hst(int b) { return *reinterpret_cast<DevState*>(h_st + SS * b); }

  ~BatchRun() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap) (void)hipStreamDestroy(cap);
    if (h_args) (void)hipHostFree(h_args);
    if (h_sw) (void)hipHostFree(h_sw);
    if (h_aw) (void)hipHostFree(h_aw);
    if (h_st) (void)hipHostFree(h_st);
  }

  // Layout and staging.  stream_mode: -1 chooses from the batch's footprint;
  // force_rows / force_per_item > 0 impose one schedule on every problem.
  int setup(drot_ctx* ctx, int32_t n, int dt, const drot_problem* ps, const drot_params* p,
            int stream_mode, int force_rows, int force_per_item, int force_chunks = 0) {
    c = ctx;
    count = n;
    dtype = dt;
    probs = ps;
    prm = *p;
    const size_t es = dtype == DROT_F32 ? 4 : 8;
    const int V = (int)(16 / es);
    bool vec_ok = true;
    double total_bytes = 0;
    for (int b = 0; b < count; ++b) {
      const drot_problem& P = probs[b];
      vec_ok = vec_ok && (uintptr_t)P.C % 16 == 0 && (uintptr_t)P.X % 16 == 0 &&
               P.ldc % V == 0 && P.ldx % V == 0;
      total_bytes += 2.0 * (double)P.m * (double)P.n * (double)es;
    }
    if (vec_ok) {
      tile.stream = stream_mode >= 0 ? stream_mode != 0
                    : prm.cache_mode == DROT_CACHE_STREAM ||
                          (prm.cache_mode == DROT_CACHE_AUTO && total_bytes > 192.0 * 1024 * 1024);
      tile.vec = V;
      // 16-byte chunks per lane: the parameter, else the tuner's choice for
      // this element type and cache policy, else 2 (512-column strips in
      // float32; measured faster than 1 on the 512-problem batch).
      const int tuned = drot_internal_batch_chunks(c, dtype * 2 + (tile.stream ? 1 : 0));
      tile.chunks = force_chunks > 0 ? force_chunks
                    : prm.tile_chunks > 0 ? prm.tile_chunks : (tuned > 0 ? tuned : 2);
      tile.ragged = true;  // masks the last chunk where n is not a multiple of V
    }
    const int64_t W = (int64_t)kWave * tile.vec * tile.chunks;

    // The device states come first, contiguous with a fixed stride, so that
    // one copy polls every problem.
    L.assign(count, ProbLayout{});
    SS = up(sizeof(DevState));
    size_t o = SS * (size_t)count;
    max_sweep = max_aux = 0;
    for (int b = 0; b < count; ++b) {
      const drot_problem& P = probs[b];
      // Untuned: 16-row blocks, one per work item (measured best among the
      // uniform schedules on the 512-problem batch).
      int rows = 16, per = 1;
      drot_internal_batch_tile(c, tile_key(dtype, tile.stream, P.m, P.n), &rows, &per);
      if (prm.tile_rows > 0) rows = prm.tile_rows;
      if (force_rows > 0) rows = force_rows;
      if (force_per_item > 0) per = force_per_item;
      SweepGeom& g = L[b].g;
      g.m = P.m;
      g.n = P.n;
      g.ldc = P.ldc;
      g.ldx = P.ldx;
      g.n_ct = (int)((P.n + W - 1) / W);
      g.rows = rows;
      g.n_rb = (int)((P.m + g.rows - 1) / g.rows);
      g.n_rg = prm.tile_groups > 0 ? std::min(prm.tile_groups, g.n_rb)
                                   : (int)((g.n_rb + per - 1) / per);
      g.ldcp = (int64_t)g.n_ct * W;
      const size_t sizes[12] = {0,
                                sizeof(double) * kBatchTrace * kTraceWidth,
                                sizeof(double) * (size_t)g.n_rg * (size_t)g.ldcp,
                                sizeof(double) * (size_t)g.n_ct * (size_t)P.m,
                                sizeof(double) * (size_t)g.n_ct * g.n_rg * kTileSlots,
                                sizeof(double) * (size_t)P.m,
                                sizeof(double) * (size_t)P.n,
                                sizeof(double) * (size_t)P.m,
                                sizeof(double) * (size_t)P.n,
                                sizeof(double) * (size_t)P.m,
                                sizeof(double) * (size_t)P.n,
                                sizeof(double) * (size_t)aux_workgroups(P.m, P.n) * kSlots};
      for (int k = 0; k < 12; ++k) {
        L[b].off[k] = o;
        o += up(sizes[k]);
      }
      max_sweep += (int64_t)g.n_ct * g.n_rg;
      max_aux += aux_workgroups(P.m, P.n);
    }
    off_args = o;
    o += up(sizeof(SweepArgs) * (size_t)count);
    off_sw = o;
    o += up(sizeof(uint2) * (size_t)max_sweep);
    off_aw = o;
    o += up(sizeof(uint2) * (size_t)max_aux);
    total = o;

    wall_rate = drot_internal_wall_rate(c);
    void* ws = nullptr;
    int rc = drot_internal_ctx_prepare(c, &ws, total);
    if (rc) return rc;
    base = static_cast<char*>(ws);
    BHIP(hipHostMalloc((void**)&h_args, sizeof(SweepArgs) * count, hipHostMallocDefault));
    BHIP(hipHostMalloc((void**)&h_sw, sizeof(uint2) * std::max<int64_t>(1, max_sweep), hipHostMallocDefault));
    BHIP(hipHostMalloc((void**)&h_aw, sizeof(uint2) * std::max<int64_t>(1, max_aux), hipHostMallocDefault));
    BHIP(hipHostMalloc((void**)&h_st, SS * count, hipHostMallocDefault));
    BHIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    for (int b = 0; b < count; ++b) {
      const drot_problem& P = probs[b];
      SweepArgs& a = h_args[b];
      a = SweepArgs{};
      a.cost_kind = kCostDense;
      a.C = P.C;
      a.X = P.X;
      a.p = P.p;
      a.q = P.q;
      a.st = reinterpret_cast<DevState*>(base + SS * b);
      a.trace = reinterpret_cast<double*>(base + L[b].off[1]);
      a.trace_cap = kBatchTrace;
      a.colpart = base + L[b].off[2];
      a.rowpart = base + L[b].off[3];
      a.tiles = reinterpret_cast<double*>(base + L[b].off[4]);
      a.a = reinterpret_cast<double*>(base + L[b].off[5]);
      a.b = reinterpret_cast<double*>(base + L[b].off[6]);
      a.phi64 = reinterpret_cast<double*>(base + L[b].off[7]);
      a.psi64 = reinterpret_cast<double*>(base + L[b].off[8]);
      a.phiT = base + L[b].off[9];
      a.psiT = base + L[b].off[10];
      a.blockpart = reinterpret_cast<double*>(base + L[b].off[11]);
      a.mu_out = P.mu;
      a.nu_out = P.nu;
      a.mu0 = P.mu0;
      a.nu0 = P.nu0;
      a.wall_rate = wall_rate;
      a.g = L[b].g;
      DevState& h = hst(b);
      memset(&h, 0, sizeof(DevState));
      h.rho = P.rho;
      h.tol = P.tol;
      h.max_iter = prm.max_iter;
      h.tol_mode = prm.tol_mode;
      h.m = P.m;
      h.n = P.n;
    }
    active.assign(count, 1);
    return DROT_OK;
  }

  const SweepArgs* d_args() const { return reinterpret_cast<const SweepArgs*>(base + off_args); }
  uint2* d_sw() const { return reinterpret_cast<uint2*>(base + off_sw); }
  uint2* d_aw() const { return reinterpret_cast<uint2*>(base + off_aw); }

  // Work lists of the problems still running (all of them when `all`).
  void build_lists(bool all) {
    n_sw = 0;
    n_aw = 0;
    for (int b = 0; b < count; ++b) {
      if (!all && !active[b]) continue;
      const int64_t nt = (int64_t)L[b].g.n_ct * L[b].g.n_rg;
      for (int64_t t = 0; t < nt; ++t) h_sw[n_sw++] = uint2{(unsigned)b, (unsigned)t};
      const int64_t na = aux_workgroups(L[b].g.m, L[b].g.n);
      for (int64_t t = 0; t < na; ++t) h_aw[n_aw++] = uint2{(unsigned)b, (unsigned)t};
    }
  }

  int upload_lists(hipStream_t s) {
    BHIP(hipMemcpyAsync(d_sw(), h_sw, sizeof(uint2) * n_sw, hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(d_aw(), h_aw, sizeof(uint2) * n_aw, hipMemcpyHostToDevice, s));
    return DROT_OK;
  }

  // Initialisation of every problem and the data checks.
  int init(hipStream_t s) {
    BHIP(hipMemcpyAsync(base, h_st, SS * count, hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(base + off_args, h_args, sizeof(SweepArgs) * count, hipMemcpyHostToDevice, s));
    build_lists(true);
    int rc = upload_lists(s);
    if (rc) return rc;
    BHIP(launch_prep_batch(d_args(), count, s));
    BHIP(launch_batch_step(dtype, kInitPQ, tile, d_args(), d_sw(), n_sw, d_aw(), n_aw, count, s));
    BHIP(hipMemcpyAsync(h_st, base, SS * count, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    const double eps = dtype == DROT_F32 ? 1.1920929e-07 : 2.220446049250313e-16;
    for (int b = 0; b < count; ++b) {
      const DevState& h = hst(b);
      if (h.init_bad > 0)
        return bfail(DROT_ENONFINITE, "problem %d: non-finite entries in C, p, q or the warm start", b);
      if (h.init_neg > 0 || !(h.sum_p > 0) ||
          std::fabs(h.sum_p - h.sum_q) > 8.0 * eps * std::max(h.sum_p, h.sum_q))
        return bfail(DROT_EMASS, "problem %d: negative marginals or unequal mass", b);
    }
    return DROT_OK;
  }

  // One group of G iterations of the live problems (a graph replay, or
  // eager launches), without waiting.
  int group(hipStream_t s, int G) {
    if (prm.flags & DROT_FLAG_NO_GRAPH) {
      build_lists(false);
      int rc = upload_lists(s);
      if (rc) return rc;
      for (int k = 0; k < G; ++k)
        BHIP(launch_batch_step(dtype, kIter, tile, d_args(), d_sw(), n_sw, d_aw(), n_aw, count, s));
      return DROT_OK;
    }
    if (!gexec) {
      build_lists(false);
      int rc = upload_lists(s);
      if (rc) return rc;
      BHIP(hipStreamSynchronize(s));
      hipGraph_t graph = nullptr;
      BHIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      hipError_t le = hipSuccess;
      for (int k = 0; k < G && le == hipSuccess; ++k)
        le = launch_batch_step(dtype, kIter, tile, d_args(), d_sw(), n_sw, d_aw(), n_aw, count, cap);
      hipError_t ee = hipStreamEndCapture(cap, &graph);
      if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bfail(DROT_EDEVICE, "batched capture: %s",
                     hipGetErrorString(le != hipSuccess ? le : ee));
      }
      hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        gexec = nullptr;
        return bfail(DROT_EDEVICE, "batched graph: %s", hipGetErrorString(ie));
      }
      grid_sw = n_sw;
    }
    BHIP(hipGraphLaunch(gexec, s));
    return DROT_OK;
  }

  // Groups until every problem has stopped (its test or max_iter); finished
  // problems leave the lists once they hold half of the captured grid.
  int run(hipStream_t s, int G) {
    int n_active = count;
    while (n_active > 0) {
      int rc = group(s, G);
      if (rc) return rc;
      BHIP(hipMemcpyAsync(h_st, base, SS * count, hipMemcpyDeviceToHost, s));
      BHIP(hipStreamSynchronize(s));
      int64_t live_tiles = 0;
      n_active = 0;
      for (int b = 0; b < count; ++b) {
        if (active[b] && hst(b).done) active[b] = 0;
        if (active[b]) {
          ++n_active;
          live_tiles += (int64_t)L[b].g.n_ct * L[b].g.n_rg;
        }
      }
      if (gexec && n_active > 0 && 2 * live_tiles < grid_sw) {
        (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
      }
    }
    return DROT_OK;
  }

  // The final FP64 evaluation of every problem.
  int final_pass(hipStream_t s) {
    build_lists(true);
    int rc = upload_lists(s);
    if (rc) return rc;
    BHIP(launch_batch_step(dtype, kFinal, tile, d_args(), d_sw(), n_sw, d_aw(), n_aw, count, s));
    BHIP(hipMemcpyAsync(h_st, base, SS * count, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    return DROT_OK;
  }

  int results(drot_result* outs, double secs) {
    int worst = DROT_OK;
    for (int b = 0; b < count; ++b) {
      const DevState& h = hst(b);
      drot_result& r = outs[b];
      memset(&r, 0, sizeof(r));
      r.iters = h.iter;
      r.status = h.done ? h.status : DROT_MAXITER;
      r.objective = h.f_pobj;
      r.dual_objective = h.f_dobj;
      r.r_primal = h.f_rp;
      r.r_dual = h.f_rd;
      r.gap = h.f_gap;
      r.eps_primal = h.f_eps_p;
      r.eps_dual = h.f_eps_d;
      r.eps_gap = h.f_eps_g;
      r.seconds_to_tol = (double)((h.done ? h.t_stop : h.t_last) - h.t_start) / wall_rate;
      r.seconds_total = secs;
      if (r.status == -3) worst = DROT_ENONFINITE;
      else if (r.status == DROT_MAXITER && worst == DROT_OK) worst = DROT_MAXITER;
    }
    if (worst == DROT_ENONFINITE) bfail(worst, "a problem of the batch produced a non-finite value");
    return worst;
  }
};

}  // namespace

extern "C" int drot_solve_batched(drot_ctx* c, int32_t count, int dtype, const drot_problem* probs,
                                  const drot_params* prm, drot_result* outs, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = validate_batch(count, dtype, probs, prm);
  if (rc) return rc;
  if (!outs) return bfail(DROT_EINVAL, "outs must be non-NULL");
  if (!c) return bfail(DROT_EINVAL, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  BatchRun r;
  if ((rc = r.setup(c, count, dtype, probs, prm, -1, 0, 0))) return rc;
  if ((rc = r.init(s))) return rc;
  const int G = prm->check_every > 0 ? prm->check_every : 32;
  if ((rc = r.run(s, G))) return rc;
  if ((rc = r.final_pass(s))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return r.results(outs, secs);
}

namespace {

// Time `groups` graph replays of G iterations of the batch (after one warm
// replay) with the schedules the context's cache holds.
int time_batch(drot_ctx* c, int32_t count, int dtype, const drot_problem* probs,
               const drot_params* trial, int stream_mode, int G, int groups, hipStream_t s,
               hipEvent_t e0, hipEvent_t e1, double* us_per_iter) {
  BatchRun r;
  int rc = r.setup(c, count, dtype, probs, trial, stream_mode, 0, 0);
  if (!rc) rc = r.init(s);
  if (!rc) rc = r.group(s, G);
  if (rc) return rc;
  BHIP(hipEventRecord(e0, s));
  for (int k = 0; k < groups && !rc; ++k) rc = r.group(s, G);
  if (rc) return rc;
  float ms = 0.f;
  BHIP(hipEventRecord(e1, s));
  BHIP(hipEventSynchronize(e1));
  BHIP(hipEventElapsedTime(&ms, e0, e1));
  *us_per_iter = ms * 1e3 / ((double)groups * G);
  return DROT_OK;
}

}  // namespace

extern "C" int drot_tune_batched(drot_ctx* c, int32_t count, int dtype, const drot_problem* probs,
                                 const drot_params* prm, int64_t iters, drot_batch_tile* table,
                                 int32_t table_cap, int32_t* n_entries, void* stream) {
  int rc = validate_batch(count, dtype, probs, prm);
  if (rc) return rc;
  if (!c) return bfail(DROT_EINVAL, "ctx is NULL");
  if (iters < 0) return bfail(DROT_EINVAL, "iters must be >= 0");
  if (table_cap < 0 || (table_cap > 0 && !table))
    return bfail(DROT_EINVAL, "table must hold table_cap entries");
  hipStream_t s = (hipStream_t)stream;
  const int G = prm->check_every > 0 ? prm->check_every : 32;
  if (iters == 0) iters = 2 * G;
  const int groups = (int)((iters + G - 1) / G);
  // The cache policy of the whole batch (the schedules are tuned under it).
  const size_t es = dtype == DROT_F32 ? 4 : 8;
  double total_bytes = 0;
  std::vector<double> class_entries(36, 0.0);
  std::vector<int> class_count(36, 0);
  for (int b = 0; b < count; ++b) {
    total_bytes += 2.0 * (double)probs[b].m * (double)probs[b].n * (double)es;
    const int k = side_bucket(probs[b].m) * 6 + side_bucket(probs[b].n);
    class_entries[k] += (double)probs[b].m * (double)probs[b].n;
    class_count[k] += 1;
  }
  const bool stream_mode = prm->cache_mode == DROT_CACHE_STREAM ||
                           (prm->cache_mode == DROT_CACHE_AUTO && total_bytes > 192.0 * 1024 * 1024);
  const int base_key = (dtype * 2 + (stream_mode ? 1 : 0)) * 36;
  // Fixed iteration counts: every problem's tolerance 0.
  std::vector<drot_problem> ps(probs, probs + count);
  for (auto& P : ps) P.tol = 0.0;
  drot_params trial = *prm;
  trial.tol_mode = DROT_TOL_ABSOLUTE;
  trial.max_iter = (int64_t)(groups + 2) * G + 1;
  trial.flags &= ~DROT_FLAG_NO_GRAPH;
  trial.tile_rows = 0;
  trial.tile_groups = 0;
  trial.tile_chunks = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(DROT_EDEVICE, "hipEventCreate failed");
  }
  auto set_all = [&](int rows, int per) {
    for (int k = 0; k < 36; ++k) drot_internal_set_batch_tile(c, base_key + k, rows, per);
  };
  // Stage 1: one schedule for every class, and the chunks per lane.
  static const int kChunks[] = {1, 2};
  static const int kRows[] = {8, 16, 32};
  static const int kPer1[] = {1, 2};
  double best = -1.0;
  int best_ch = 2, best_rows = 16, best_per = 1;
  for (int ch : kChunks)
    for (int rows : kRows)
      for (int per : kPer1) {
        if (rc) break;
        set_all(rows, per);
        drot_internal_set_batch_chunks(c, dtype * 2 + (stream_mode ? 1 : 0), ch);
        double us = 0.0;
        rc = time_batch(c, count, dtype, ps.data(), &trial, stream_mode ? 1 : 0, G, groups, s, e0,
                        e1, &us);
        if (!rc && (best < 0 || us < best)) {
          best = us;
          best_ch = ch;
          best_rows = rows;
          best_per = per;
        }
      }
  set_all(best_rows, best_per);
  drot_internal_set_batch_chunks(c, dtype * 2 + (stream_mode ? 1 : 0), best_ch);
  // Stage 2: each class holding at least 5% of the entries, largest first,
  // with the others fixed; a change is kept when it is 1% faster.
  std::vector<int> order;
  double all_entries = 0;
  for (int k = 0; k < 36; ++k) all_entries += class_entries[k];
  for (int k = 0; k < 36; ++k)
    if (class_entries[k] >= 0.05 * all_entries) order.push_back(k);
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return class_entries[x] > class_entries[y]; });
  static const int kPer2[] = {1, 2, 4};
  for (int k : order) {
    int cur_rows = best_rows, cur_per = best_per;
    drot_internal_batch_tile(c, base_key + k, &cur_rows, &cur_per);
    for (int rows : kRows)
      for (int per : kPer2) {
        if (rc || (rows == cur_rows && per == cur_per)) continue;
        drot_internal_set_batch_tile(c, base_key + k, rows, per);
        double us = 0.0;
        rc = time_batch(c, count, dtype, ps.data(), &trial, stream_mode ? 1 : 0, G, groups, s, e0,
                        e1, &us);
        if (!rc && us < 0.99 * best) {
          best = us;
          cur_rows = rows;
          cur_per = per;
        }
        drot_internal_set_batch_tile(c, base_key + k, cur_rows, cur_per);
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  int32_t entries = 0;
  for (int k = 0; k < 36; ++k) {
    if (!class_count[k]) continue;
    if (entries < table_cap) {
      int rows = 0, per = 0;
      drot_internal_batch_tile(c, base_key + k, &rows, &per);
      drot_batch_tile& t = table[entries];
      t.m_class = k / 6;
      t.n_class = k % 6;
      t.tile_rows = rows;
      t.blocks_per_item = per;
      t.problems = class_count[k];
      t.chunks = best_ch;
      t.us_per_iter = best;
    }
    ++entries;
  }
  if (n_entries) *n_entries = entries;
  return DROT_OK;
}
