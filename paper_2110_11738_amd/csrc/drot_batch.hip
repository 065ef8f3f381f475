// Host side of the batched solver: many independent OT problems of different
// shapes advance together, one batched sweep launch and one batched aux launch
// per iteration over work lists of (problem, workgroup) pairs.  Every problem
// keeps its own device state and stopping test (Algorithm 1 and the stopping
// criteria of Section 3, per problem); finished problems are dropped from the
// work lists when the lists are rebuilt.
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
    if (e_ != hipSuccess) {                                                          \
      rc = bfail(DROT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
      goto done;                                                                     \
    }                                                                                \
  } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr int kBatchTrace = 256;

struct ProbLayout {
  SweepGeom g;
  size_t off[12];
};

}  // namespace

extern "C" int drot_solve_batched(drot_ctx* c, int32_t count, int dtype, const drot_problem* probs,
                                  const drot_params* prm, drot_result* outs, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (count < 1) return bfail(DROT_EINVAL, "count must be >= 1");
  if (!probs || !prm || !outs) return bfail(DROT_EINVAL, "probs, params and outs must be non-NULL");
  if (dtype != DROT_F32 && dtype != DROT_F64) return bfail(DROT_EINVAL, "unknown dtype %d", dtype);
  if (!(prm->max_iter >= 1)) return bfail(DROT_EINVAL, "max_iter must be >= 1");
  if (prm->tol_mode != DROT_TOL_RELATIVE && prm->tol_mode != DROT_TOL_ABSOLUTE)
    return bfail(DROT_EINVAL, "unknown tol_mode %d", prm->tol_mode);
  if (prm->flags & ~(DROT_FLAG_NO_GRAPH))
    return bfail(DROT_EUNSUPPORTED, "batched solves take only DROT_FLAG_NO_GRAPH");
  if (prm->tile_chunks < 0 || prm->tile_chunks > 2 || prm->tile_rows < 0 || prm->tile_rows > 4096)
    return bfail(DROT_EINVAL, "bad tile parameters");
  const size_t es = dtype == DROT_F32 ? 4 : 8;
  const int V = (int)(16 / es);

  // ---- validation and the shared tile variant ------------------------------
  bool vec_ok = true;
  double total_bytes = 0;
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
    vec_ok = vec_ok && (uintptr_t)P.C % 16 == 0 && (uintptr_t)P.X % 16 == 0 && P.ldc % V == 0 &&
             P.ldx % V == 0;
    total_bytes += 2.0 * (double)P.m * (double)P.n * (double)es;
  }
  if (!c) return bfail(DROT_EINVAL, "ctx is NULL");
  TileCfg tile{1, 4, 4, false, false};
  if (vec_ok) {
    tile.stream = prm->cache_mode == DROT_CACHE_STREAM ||
                  (prm->cache_mode == DROT_CACHE_AUTO && total_bytes > 192.0 * 1024 * 1024);
    tile.vec = V;
    tile.chunks = prm->tile_chunks > 0 ? prm->tile_chunks : 1;
    tile.ragged = true;  // masks the last chunk where n is not a multiple of V
  }
  const int64_t W = (int64_t)kWave * tile.vec * tile.chunks;
  const int rows_default = prm->tile_rows > 0 ? prm->tile_rows : (tile.stream ? 16 : 32);

  // ---- workspace layout -----------------------------------------------------
  // The device states come first, contiguous with a fixed stride, so that one
  // copy polls every problem.
  std::vector<ProbLayout> L(count);
  const size_t SS = up(sizeof(DevState));
  size_t o = SS * (size_t)count;
  int64_t max_sweep = 0, max_aux = 0;
  for (int b = 0; b < count; ++b) {
    const drot_problem& P = probs[b];
    SweepGeom& g = L[b].g;
    g.m = P.m;
    g.n = P.n;
    g.ldc = P.ldc;
    g.ldx = P.ldx;
    g.n_ct = (int)((P.n + W - 1) / W);
    g.rows = rows_default;
    g.n_rb = (int)((P.m + g.rows - 1) / g.rows);
    g.n_rg = g.n_rb;
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
  const size_t off_args = o;
  o += up(sizeof(SweepArgs) * (size_t)count);
  const size_t off_sw = o;
  o += up(sizeof(uint2) * (size_t)max_sweep);
  const size_t off_aw = o;
  o += up(sizeof(uint2) * (size_t)max_aux);
  const size_t total = o;

  int rc = DROT_OK;
  void* ws = nullptr;
  char* base = nullptr;
  hipStream_t s = (hipStream_t)stream;
  // Pinned staging for the args, the work lists and the device states.
  SweepArgs* h_args = nullptr;
  uint2* h_sw = nullptr;
  uint2* h_aw = nullptr;
  char* h_st = nullptr;  // count records with stride SS
  auto hst = [&](int b) -> DevState& { return *reinterpret_cast<DevState*>(h_st + SS * b); };
  hipGraphExec_t gexec = nullptr;
  int g_iters = 0;
  int64_t n_sw = 0, n_aw = 0;
  std::vector<char> active(count, 1);
  const int G = prm->check_every > 0 ? prm->check_every : 32;
  const double wall_rate = drot_internal_wall_rate(c);
  hipStream_t cap = nullptr;

  if ((rc = drot_internal_ctx_prepare(c, &ws, total))) return rc;
  base = static_cast<char*>(ws);
  BHIP(hipHostMalloc((void**)&h_args, sizeof(SweepArgs) * count, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_sw, sizeof(uint2) * std::max<int64_t>(1, max_sweep), hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_aw, sizeof(uint2) * std::max<int64_t>(1, max_aux), hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&h_st, SS * count, hipHostMallocDefault));
  BHIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));

  for (int b = 0; b < count; ++b) {
    const drot_problem& P = probs[b];
    char* pb = base;
    SweepArgs& a = h_args[b];
    a = SweepArgs{};
    a.cost_kind = kCostDense;
    a.C = P.C;
    a.X = P.X;
    a.p = P.p;
    a.q = P.q;
    a.st = reinterpret_cast<DevState*>(pb + SS * b);
    a.trace = reinterpret_cast<double*>(pb + L[b].off[1]);
    a.trace_cap = kBatchTrace;
    a.colpart = pb + L[b].off[2];
    a.rowpart = pb + L[b].off[3];
    a.tiles = reinterpret_cast<double*>(pb + L[b].off[4]);
    a.a = reinterpret_cast<double*>(pb + L[b].off[5]);
    a.b = reinterpret_cast<double*>(pb + L[b].off[6]);
    a.phi64 = reinterpret_cast<double*>(pb + L[b].off[7]);
    a.psi64 = reinterpret_cast<double*>(pb + L[b].off[8]);
    a.phiT = pb + L[b].off[9];
    a.psiT = pb + L[b].off[10];
    a.blockpart = reinterpret_cast<double*>(pb + L[b].off[11]);
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
    h.max_iter = prm->max_iter;
    h.tol_mode = prm->tol_mode;
    h.m = P.m;
    h.n = P.n;
  }
  {
    const SweepArgs* d_args = reinterpret_cast<const SweepArgs*>(base + off_args);
    uint2* d_sw = reinterpret_cast<uint2*>(base + off_sw);
    uint2* d_aw = reinterpret_cast<uint2*>(base + off_aw);

    // Work lists of the problems still running (all of them for init/final).
    auto build_lists = [&](bool all) {
      n_sw = 0;
      n_aw = 0;
      for (int b = 0; b < count; ++b) {
        if (!all && !active[b]) continue;
        const int64_t nt = (int64_t)L[b].g.n_ct * L[b].g.n_rg;
        for (int64_t t = 0; t < nt; ++t) h_sw[n_sw++] = uint2{(unsigned)b, (unsigned)t};
        const int64_t na = aux_workgroups(L[b].g.m, L[b].g.n);
        for (int64_t t = 0; t < na; ++t) h_aw[n_aw++] = uint2{(unsigned)b, (unsigned)t};
      }
    };

    BHIP(hipMemcpyAsync(base, h_st, SS * count, hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(base + off_args, h_args, sizeof(SweepArgs) * count, hipMemcpyHostToDevice, s));
    build_lists(true);
    BHIP(hipMemcpyAsync(d_sw, h_sw, sizeof(uint2) * n_sw, hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(d_aw, h_aw, sizeof(uint2) * n_aw, hipMemcpyHostToDevice, s));
    BHIP(launch_prep_batch(d_args, count, s));
    BHIP(launch_batch_step(dtype, kInitPQ, tile, d_args, d_sw, n_sw, d_aw, n_aw, count, s));
    BHIP(hipMemcpyAsync(h_st, base, SS * count, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    const double eps = dtype == DROT_F32 ? 1.1920929e-07 : 2.220446049250313e-16;
    for (int b = 0; b < count; ++b) {
      const DevState& h = hst(b);
      if (h.init_bad > 0) {
        rc = bfail(DROT_ENONFINITE, "problem %d: non-finite entries in C, p, q or the warm start", b);
        goto done;
      }
      if (h.init_neg > 0 || !(h.sum_p > 0) ||
          std::fabs(h.sum_p - h.sum_q) > 8.0 * eps * std::max(h.sum_p, h.sum_q)) {
        rc = bfail(DROT_EMASS, "problem %d: negative marginals or unequal mass", b);
        goto done;
      }
    }

    // ---- iterations -----------------------------------------------------------
    int64_t grid_sw = 0;  // sweep work items the current graph was built for
    int n_active = count;
    while (n_active > 0) {
      if (!(prm->flags & DROT_FLAG_NO_GRAPH)) {
        if (!gexec) {
          build_lists(false);
          BHIP(hipMemcpyAsync(d_sw, h_sw, sizeof(uint2) * n_sw, hipMemcpyHostToDevice, s));
          BHIP(hipMemcpyAsync(d_aw, h_aw, sizeof(uint2) * n_aw, hipMemcpyHostToDevice, s));
          BHIP(hipStreamSynchronize(s));
          hipGraph_t graph = nullptr;
          BHIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
          hipError_t le = hipSuccess;
          for (int k = 0; k < G && le == hipSuccess; ++k)
            le = launch_batch_step(dtype, kIter, tile, d_args, d_sw, n_sw, d_aw, n_aw, count, cap);
          hipError_t ee = hipStreamEndCapture(cap, &graph);
          if (le != hipSuccess || ee != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            rc = bfail(DROT_EDEVICE, "batched capture: %s",
                       hipGetErrorString(le != hipSuccess ? le : ee));
            goto done;
          }
          hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          if (ie != hipSuccess) {
            gexec = nullptr;
            rc = bfail(DROT_EDEVICE, "batched graph: %s", hipGetErrorString(ie));
            goto done;
          }
          g_iters = G;
          grid_sw = n_sw;
        }
        BHIP(hipGraphLaunch(gexec, s));
      } else {
        build_lists(false);
        BHIP(hipMemcpyAsync(d_sw, h_sw, sizeof(uint2) * n_sw, hipMemcpyHostToDevice, s));
        BHIP(hipMemcpyAsync(d_aw, h_aw, sizeof(uint2) * n_aw, hipMemcpyHostToDevice, s));
        for (int k = 0; k < G; ++k)
          BHIP(launch_batch_step(dtype, kIter, tile, d_args, d_sw, n_sw, d_aw, n_aw, count, s));
      }
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
      // Drop finished problems from the lists once they hold half the grid.
      if (gexec && n_active > 0 && 2 * live_tiles < grid_sw) {
        (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
      }
    }
    (void)g_iters;

    // ---- final evaluation of every problem --------------------------------------
    build_lists(true);
    BHIP(hipMemcpyAsync(d_sw, h_sw, sizeof(uint2) * n_sw, hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(d_aw, h_aw, sizeof(uint2) * n_aw, hipMemcpyHostToDevice, s));
    BHIP(launch_batch_step(dtype, kFinal, tile, d_args, d_sw, n_sw, d_aw, n_aw, count, s));
    BHIP(hipMemcpyAsync(h_st, base, SS * count, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
  }
  {
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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
    rc = worst;
    if (rc == DROT_ENONFINITE) bfail(rc, "a problem of the batch produced a non-finite value");
  }
done:
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (cap) (void)hipStreamDestroy(cap);
  if (h_args) (void)hipHostFree(h_args);
  if (h_sw) (void)hipHostFree(h_sw);
  if (h_aw) (void)hipHostFree(h_aw);
  if (h_st) (void)hipHostFree(h_st);
  return rc;
}
