// Host side of libdrot.so: the C ABI of include/drot.h.
//
// Validation, the per-context workspace, the iteration driver (hipGraphs of
// `check_every` iterations replayed on the caller's stream, early exit on the
// device stop flag), polling, the final evaluation and error reporting.
// Every computation of the method runs in the kernels of drot_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/drot.h"
#include "drot_internal.h"

using namespace drot;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(DROT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Geometry {
  TileCfg tile{1, 1, 4, false, false};
  SweepGeom g{};
  int n_tiles = 0;
};

}  // namespace

struct drot_ctx {
  int device = 0;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  double wall_rate = 1e8;

  // Workspace (one allocation, carved up per bind).  fixed_ws: the workspace
  // is the library's static scratch (drot_solve_noalloc), never grown.
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool fixed_ws = false;
  DevState* st = nullptr;        // device
  DevState* st_host = nullptr;   // pinned mirror
  double* trace = nullptr;

  // Bound problem.
  bool bound = false;
  int dtype = 0;
  drot_params prm{};
  struct {  // the arguments of the latest drot_bind_cost (for drot_tune)
    int64_t m, n, ldx;
    drot_cost cost;
    const void *p, *q;
    void* X;
    const double *mu0, *nu0;
  } args{};
  Geometry geo;
  SweepArgs sa{};
  bool finished = false;

  // Small problems iterate in one workgroup (small_kernel) instead of
  // sweep + aux launches.
  bool small = false;
  // Pending form of the iteration (fewer than kAuxSplitMin aux workgroups):
  // the aux launch only publishes its sums and the next sweep takes the
  // scalar steps; state records st[0] (committed, what the host reads) and
  // st[1], sum buffers bp[0] and bp[1], used by step parity within a group.
  bool pend = false;
  double* bp[2] = {nullptr, nullptr};

  // Iterations enqueued since bind (the skip-C schedule alternates by parity).
  bool skipc = false;
  int64_t enq = 0;

  // Graph of `check_every` iterations.
  hipGraphExec_t gexec = nullptr;
  int g_iters = 0;
  bool g_timed = false;

  // Tuner cache of the batched solver: rows per block and row blocks per
  // work item by size-class key (drot_batch.hip), 0 = untuned.
  static constexpr int kBatchKeys = 2 * 2 * 36;
  int batch_rows[kBatchKeys] = {};
  int batch_per[kBatchKeys] = {};
  int batch_chunks[4] = {};  // by element type and cache policy

  // Sweep timing (DROT_FLAG_TIME_SWEEP).
  std::vector<hipEvent_t> ev;
  double sweep_ms = 0.0;
  int64_t sweep_n = 0;
};

namespace {

void drop_graph(drot_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->g_iters = 0;
}

int choose_geometry(int dtype, int64_t m, int64_t n, const drot_cost* cost, const void* X,
                    int64_t ldx, const drot_params* p, Geometry* out) {
  const size_t es = dtype == DROT_F32 ? 4 : 8;
  const int V = (int)(16 / es);
  // 16-byte path: X (and a dense C) 16-byte aligned with leading dimensions
  // that are multiples of the vector width; n itself may be ragged.
  bool aligned = ((uintptr_t)X % 16 == 0) && (ldx % V == 0);
  if (cost->kind == DROT_COST_DENSE)
    aligned = aligned && ((uintptr_t)cost->data % 16 == 0) && (cost->ld % V == 0);
  if (cost->kind == DROT_COST_BF16)
    aligned = aligned && ((uintptr_t)cost->data % 8 == 0) && (cost->ld % V == 0);
  if (p->tile_chunks < 0 || p->tile_chunks > 2)
    return fail(DROT_EINVAL, "tile_chunks must be 0, 1 or 2 (got %d)", p->tile_chunks);
  if (p->tile_unroll != 0 && p->tile_unroll != 4 && p->tile_unroll != 8)
    return fail(DROT_EINVAL, "tile_unroll must be 0, 4 or 8 (got %d)", p->tile_unroll);
  if (p->cache_mode < DROT_CACHE_AUTO || p->cache_mode > DROT_CACHE_STREAM)
    return fail(DROT_EINVAL, "unknown cache_mode %d", p->cache_mode);
  Geometry g;
  const double cbytes = cost->kind == DROT_COST_DENSE ? (double)es
                        : cost->kind == DROT_COST_BF16 ? 2.0 : 0.0;
  const double bytes = (double)m * (double)n * ((double)es + cbytes);
  g.tile.comp = (p->flags & DROT_FLAG_COMPENSATED) && dtype == DROT_F32;
  // The compensated iteration has no masked-chunk variant: ragged widths take
  // the scalar path.
  if (g.tile.comp && n % V != 0) aligned = false;
  if (aligned) {
    // Measured on MI355X: while X and C fit in the last-level cache, cached
    // accesses with 2 chunks per lane and 32-row blocks; above it, streaming
    // accesses with 1 chunk per lane and 16-row blocks.
    g.tile.vec = V;
    g.tile.stream = p->cache_mode == DROT_CACHE_STREAM ||
                    (p->cache_mode == DROT_CACHE_AUTO && bytes > 192.0 * 1024 * 1024);
    g.tile.chunks = p->tile_chunks > 0 ? p->tile_chunks : (g.tile.stream ? 1 : 2);
    g.tile.unroll = p->tile_unroll > 0 ? p->tile_unroll : 4;
    g.tile.ragged = n % V != 0;
    if (g.tile.ragged || g.tile.comp) g.tile.unroll = 4;
  } else {
    // Scalar path: 4-byte/8-byte accesses, cached, 4 rows in flight.
    g.tile.vec = 1;
    g.tile.chunks = p->tile_chunks == 1 && !g.tile.comp ? 1 : 4;
    g.tile.unroll = 4;
    g.tile.stream = false;
  }
  const int64_t W = (int64_t)kWave * g.tile.vec * g.tile.chunks;
  const int64_t n_ct = (n + W - 1) / W;
  int rows = p->tile_rows;
  if (rows < 0 || rows > 4096) return fail(DROT_EINVAL, "tile_rows must be in [0, 4096]");
  if (p->tile_groups < 0) return fail(DROT_EINVAL, "tile_groups must be >= 0");
  if (rows == 0) {
    rows = g.tile.stream ? 16 : 32;
    // Small problems: shorter blocks so that 512+ workgroups share 256 CUs.
    while (rows > 4 && ((m + rows - 1) / rows) * n_ct < 512) rows /= 2;
  }
  const int64_t n_rb = (m + rows - 1) / rows;
  // Row groups (workgroups per strip).  Cached problems: one row block per
  // workgroup, which measured fastest (many short-lived workgroups keep the
  // band in flight dense).  Streamed problems: two row blocks per workgroup,
  // which measured 4-5% faster per iteration at 20000 x 20000 and halves the
  // column partials that the aux kernel reads.
  int64_t n_rg = p->tile_groups > 0 ? p->tile_groups
                 : (g.tile.vec > 1 && g.tile.stream && p->tile_rows == 0) ? (n_rb + 1) / 2
                                                                           : n_rb;
  n_rg = std::max<int64_t>(1, std::min<int64_t>(n_rg, n_rb));
  if (n_ct * n_rg > 0x7fffffffLL) return fail(DROT_EUNSUPPORTED, "too many tiles");
  g.g.m = m;
  g.g.n = n;
  g.g.ldc = cost->kind == DROT_COST_COORDS ? 0 : cost->ld;
  g.g.ldx = ldx;
  g.g.n_ct = (int)n_ct;
  g.g.n_rb = (int)n_rb;
  g.g.n_rg = (int)n_rg;
  g.g.rows = rows;
  g.g.ldcp = n_ct * W;
  g.n_tiles = (int)(n_ct * n_rg);
  *out = g;
  return DROT_OK;
}

int validate(int64_t m, int64_t n, int dtype, const drot_cost* cost, const void* p,
             const void* q, const drot_params* prm, void* X, int64_t ldx, const double* mu0,
             const double* nu0) {
  if (m < 1 || n < 1) return fail(DROT_EINVAL, "m and n must be >= 1 (got %lld, %lld)",
                                  (long long)m, (long long)n);
  if (dtype != DROT_F32 && dtype != DROT_F64) return fail(DROT_EINVAL, "unknown dtype %d", dtype);
  if (!cost) return fail(DROT_EINVAL, "cost descriptor is NULL");
  if (cost->kind < DROT_COST_DENSE || cost->kind > DROT_COST_COORDS)
    return fail(DROT_EINVAL, "unknown cost kind %d", cost->kind);
  if (cost->kind != DROT_COST_COORDS && cost->ld < n)
    return fail(DROT_EINVAL, "leading dimensions must be >= n");
  if (ldx < n) return fail(DROT_EINVAL, "leading dimensions must be >= n");
  if (!prm) return fail(DROT_EINVAL, "params is NULL");
  if (!(prm->rho > 0) || !std::isfinite(prm->rho))
    return fail(DROT_EINVAL, "rho must be positive and finite");
  if (!(prm->tol >= 0) || !std::isfinite(prm->tol))
    return fail(DROT_EINVAL, "tol must be >= 0 and finite");
  if (prm->max_iter < 1) return fail(DROT_EINVAL, "max_iter must be >= 1");
  if (prm->tol_mode != DROT_TOL_RELATIVE && prm->tol_mode != DROT_TOL_ABSOLUTE)
    return fail(DROT_EINVAL, "unknown tol_mode %d", prm->tol_mode);
  if (prm->x0_mode != DROT_X0_PQ && prm->x0_mode != DROT_X0_GIVEN)
    return fail(DROT_EINVAL, "unknown x0_mode %d", prm->x0_mode);
  if (prm->check_every < 0) return fail(DROT_EINVAL, "check_every must be >= 0");
  if (prm->flags &
      ~(DROT_FLAG_NO_GRAPH | DROT_FLAG_TIME_SWEEP | DROT_FLAG_SKIP_C | DROT_FLAG_COMPENSATED))
    return fail(DROT_EINVAL, "unknown flags 0x%x", prm->flags);
  if ((prm->flags & DROT_FLAG_SKIP_C) && (prm->flags & DROT_FLAG_COMPENSATED))
    return fail(DROT_EUNSUPPORTED, "the skip-C schedule has no compensated variant");
  if (cost->kind != DROT_COST_DENSE && dtype != DROT_F32)
    return fail(DROT_EUNSUPPORTED, "bfloat16 and coordinate costs need a float32 problem");
  if (cost->kind != DROT_COST_DENSE && (prm->flags & DROT_FLAG_SKIP_C))
    return fail(DROT_EUNSUPPORTED, "the skip-C schedule needs a dense cost matrix");
  if (cost->kind == DROT_COST_COORDS) {
    if (cost->dim < 1 || cost->dim > 3) return fail(DROT_EINVAL, "coordinate dimension must be 1..3");
    if (!cost->xs || !cost->xt) return fail(DROT_EINVAL, "xs and xt must be non-NULL");
    if ((uintptr_t)cost->xs % 4 || (uintptr_t)cost->xt % 4)
      return fail(DROT_EINVAL, "coordinates must be 4-byte aligned");
    if (!(cost->scale >= 0) || !std::isfinite(cost->scale))
      return fail(DROT_EINVAL, "scale must be >= 0 and finite");
  } else if (!cost->data) {
    return fail(DROT_EINVAL, "C must be non-NULL");
  }
  const void* C = cost->kind == DROT_COST_COORDS ? nullptr : cost->data;
  const int64_t ldc = cost->ld;
  if (!p || !q || !X) return fail(DROT_EINVAL, "C, p, q and X must be non-NULL");
  if ((mu0 == nullptr) != (nu0 == nullptr))
    return fail(DROT_EINVAL, "mu0 and nu0 must be given together");
  const size_t es = dtype == DROT_F32 ? 4 : 8;
  const size_t ces = cost->kind == DROT_COST_BF16 ? 2 : es;
  if ((C && (uintptr_t)C % ces) || (uintptr_t)X % es || (uintptr_t)p % es || (uintptr_t)q % es)
    return fail(DROT_EINVAL, "arrays must be aligned to their element size");
  if (C) {
    // Overlap of C and X (both m x n with their leading dimensions).
    const uintptr_t c0 = (uintptr_t)C, c1 = c0 + (size_t)((m - 1) * ldc + n) * ces;
    const uintptr_t x0 = (uintptr_t)X, x1 = x0 + (size_t)((m - 1) * ldx + n) * es;
    if (c0 < x1 && x0 < c1) return fail(DROT_EINVAL, "C and X overlap");
  }
  return DROT_OK;
}

// Offsets of the workspace's parts (offs[12]) and its total size.
size_t workspace_layout(int64_t m, int64_t n, const Geometry& g, size_t* offs) {
  // st, trace, colpart, rowpart, tiles, a, b, phi64, psi64, phiT, psiT,
  // blockpart
  size_t o = 0;
  const size_t sizes[12] = {
      2 * sizeof(DevState),
      sizeof(double) * kTraceCap * kTraceWidth,
      sizeof(double) * (size_t)g.g.n_rg * (size_t)g.g.ldcp,
      sizeof(double) * (size_t)g.g.n_ct * (size_t)m,
      sizeof(double) * (size_t)g.n_tiles * kTileSlots,
      sizeof(double) * (size_t)m,
      sizeof(double) * (size_t)n,
      sizeof(double) * (size_t)m,
      sizeof(double) * (size_t)n,
      sizeof(double) * (size_t)m,
      sizeof(double) * (size_t)n,
      2 * sizeof(double) * (size_t)aux_workgroups(m, n) * kSlots};
  for (int k = 0; k < 12; ++k) {
    offs[k] = o;
    o += up(sizes[k]);
  }
  return o;
}

int ensure_workspace(drot_ctx* c, int64_t m, int64_t n, const Geometry& g, size_t* offs) {
  const size_t o = workspace_layout(m, n, g, offs);
  if (o <= c->ws_bytes) return DROT_OK;
  if (c->fixed_ws)
    return fail(DROT_EINVAL,
                "a %lld x %lld problem needs %zu bytes of workspace, more than the %zu bytes of "
                "static scratch",
                (long long)m, (long long)n, o, c->ws_bytes);
  drop_graph(c);
  if (c->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  const size_t want = o + o / 4;  // headroom so that slightly larger problems reuse it
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    c->ws = nullptr;
    return fail(DROT_ENOMEM, "workspace allocation of %zu bytes failed", want);
  }
  c->ws_bytes = want;
  return DROT_OK;
}

// Sweep mode of the iteration with 0-based index `idx` since bind: plain, or
// alternating C-reading / C-free under the skip-C schedule.
int iter_mode(const drot_ctx* c, int64_t idx) {
  if (!c->skipc) return kIter;
  return (idx & 1) ? kIterB : kIterA;
}

// Kernel arguments of step j (0-based) of a group of iterations, whose first
// iteration has global index `first` (iterations enqueued since bind).  A
// group starts from the committed state in st[0].  Pending form: step j's
// sweep closes iteration j - 1 from (st[(j-1)&1], bp[(j-1)&1]) and commits
// st[j&1]; step j's aux reads st[j&1] and publishes into bp[j&1]; so no
// kernel writes a record or buffer that another of its workgroups reads.
SweepArgs step_args(const drot_ctx* c, int j, int64_t first) {
  SweepArgs a = c->sa;
  if (!c->pend) return a;
  const int cur = j & 1;
  a.st = c->st + cur;
  a.blockpart = c->bp[cur];
  if (j > 0) {
    a.st_prev = c->st + (1 - cur);
    a.bp_prev = c->bp[1 - cur];
    a.prev_b = iter_mode(c, first + j - 1) == kIterB ? 1 : 0;
  }
  return a;
}

// The finishing launch of a group of k >= 1 steps (pending form): closes the
// group's last iteration into st[0].
int launch_group_end(drot_ctx* c, hipStream_t s, int k, int64_t first) {
  if (!c->pend || k < 1) return DROT_OK;
  SweepArgs a = c->sa;
  a.st_prev = c->st + ((k - 1) & 1);
  a.bp_prev = c->bp[(k - 1) & 1];
  HIP_TRY(launch_finish(iter_mode(c, first + k - 1), a, s));
  return DROT_OK;
}

// Step j of a group: sweep + aux.  With events (eager timing) the sweep's
// start and end are the dispatch's own timestamps.
int launch_iteration(drot_ctx* c, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int j,
                     int64_t first) {
  const int mode = iter_mode(c, first + j);
  const SweepArgs a = step_args(c, j, first);
  HIP_TRY(launch_sweep(c->dtype, mode, c->geo.tile, a, s, e0, e1));
  HIP_TRY(launch_aux(c->dtype, mode, a, s, c->geo.tile.comp, c->pend));
  return DROT_OK;
}

// Iterations per graph / per host poll (even under the skip-C schedule, so
// that every graph starts with a C-reading iteration).
int group_size(const drot_ctx* c) {
  int g = c->prm.check_every > 0 ? c->prm.check_every : (c->small ? 1024 : 32);
  if (c->skipc && (g & 1)) ++g;
  return g;
}

int ensure_events(drot_ctx* c, int count) {
  while ((int)c->ev.size() < count) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  return DROT_OK;
}

// Capture one launch of step j of a group (kind 0: the sweep, 1: the aux
// kernel, 2: the group's finishing launch after j + 1 steps) into a graph.
int capture_one(drot_ctx* c, int kind, int j, int64_t first, hipGraph_t* out) {
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const int mode = iter_mode(c, first + j);
  const SweepArgs a = step_args(c, j, first);
  hipError_t e = hipSuccess;
  if (kind == 0) e = launch_sweep(c->dtype, mode, c->geo.tile, a, c->cap_stream);
  if (kind == 1) e = launch_aux(c->dtype, mode, a, c->cap_stream, c->geo.tile.comp, c->pend);
  if (kind == 2 && launch_group_end(c, c->cap_stream, j + 1, first)) e = hipErrorInvalidValue;
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(DROT_EDEVICE, "capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  *out = g;
  return DROT_OK;
}

// Position of the first timed sweep in a graph of G iterations, and the
// number of timed sweeps (DROT_FLAG_TIME_SWEEP): two consecutive sweeps in the
// middle of the graph (a C-reading and a C-free one under the skip-C
// schedule), so that timing perturbs the replay as little as possible.
int timed_first(int G) { return 2 * (G / 4); }
int timed_count(int G) { return std::min(2, G - timed_first(G)); }

// Graph of G iterations with event-record nodes around the timed sweeps,
// built node by node; the kernels enter as captured child graphs.
int build_timed_graph(drot_ctx* c, int G, hipGraph_t* out) {
  // Child graphs of the step kinds: the arguments of step k depend on k only
  // through k == 0, the parity of k (the pending form's records, the skip-C
  // schedule) and, for the finishing launch, the parity of G.
  hipGraph_t gs[3] = {nullptr, nullptr, nullptr}, ga[3] = {nullptr, nullptr, nullptr};
  hipGraph_t gf = nullptr, g = nullptr;
  int rc = DROT_OK;
  for (int q = 0; q < 3 && q < G && !rc; ++q) {
    rc = capture_one(c, 0, q, 0, &gs[q]);
    if (!rc) rc = capture_one(c, 1, q, 0, &ga[q]);
  }
  if (!rc && c->pend) rc = capture_one(c, 2, G - 1, 0, &gf);
  hipError_t e = hipSuccess;
  if (!rc) e = hipGraphCreate(&g, 0);
  hipGraphNode_t prev = nullptr;
  const int t0 = timed_first(G), tn = timed_count(G);
  for (int k = 0; k < G && !rc && e == hipSuccess; ++k) {
    const int q = k == 0 ? 0 : 2 - (k & 1);  // 0: first, 1: odd, 2: even step
    const bool timed = k >= t0 && k < t0 + tn;
    const int slot = k - t0;
    hipGraphNode_t e0 = nullptr, s = nullptr, e1 = nullptr, x = nullptr;
    const hipGraphNode_t* dep = prev ? &prev : nullptr;
    size_t ndep = prev ? 1 : 0;
    if (timed) {
      e = hipGraphAddEventRecordNode(&e0, g, dep, ndep, c->ev[2 * slot]);
      dep = &e0;
      ndep = 1;
    }
    if (e == hipSuccess) e = hipGraphAddChildGraphNode(&s, g, dep, ndep, gs[q]);
    dep = &s;
    if (timed && e == hipSuccess) {
      e = hipGraphAddEventRecordNode(&e1, g, &s, 1, c->ev[2 * slot + 1]);
      dep = &e1;
    }
    if (e == hipSuccess) e = hipGraphAddChildGraphNode(&x, g, dep, 1, ga[q]);
    prev = x;
  }
  if (!rc && e == hipSuccess && gf) {
    hipGraphNode_t f = nullptr;
    e = hipGraphAddChildGraphNode(&f, g, &prev, 1, gf);
  }
  for (int q = 0; q < 3; ++q) {
    if (gs[q]) (void)hipGraphDestroy(gs[q]);
    if (ga[q]) (void)hipGraphDestroy(ga[q]);
  }
  if (gf) (void)hipGraphDestroy(gf);
  if (!rc && e != hipSuccess) rc = fail(DROT_EDEVICE, "timed graph: %s", hipGetErrorString(e));
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc;
  }
  *out = g;
  return DROT_OK;
}

int ensure_graph(drot_ctx* c) {
  const int G = group_size(c);
  const bool timed = (c->prm.flags & DROT_FLAG_TIME_SWEEP) != 0;
  if (c->gexec && c->g_iters == G && c->g_timed == timed) return DROT_OK;
  drop_graph(c);
  hipGraph_t graph = nullptr;
  if (timed) {
    int rc = ensure_events(c, 2 * timed_count(G));
    if (rc) return rc;
    if ((rc = build_timed_graph(c, G, &graph))) return rc;
  } else {
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = DROT_OK;
    for (int k = 0; k < G && rc == DROT_OK; ++k)
      rc = launch_iteration(c, c->cap_stream, nullptr, nullptr, k, 0);
    if (rc == DROT_OK) rc = launch_group_end(c, c->cap_stream, G, 0);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc != DROT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(DROT_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  hipError_t e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return fail(DROT_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  c->g_iters = G;
  c->g_timed = timed;
  return DROT_OK;
}

int harvest_events(drot_ctx* c, int pairs) {
  for (int k = 0; k < pairs; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    c->sweep_ms += ms;
    c->sweep_n += 1;
  }
  return DROT_OK;
}

int check_ctx(drot_ctx* c) {
  if (!c) return fail(DROT_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  return DROT_OK;
}

}  // namespace

// Helpers for the batched driver (drot_batch.hip).
int drot_internal_fail(int code, const char* msg) { return fail(code, "%s", msg); }

double drot_internal_wall_rate(const drot_ctx* c) { return c->wall_rate; }

bool drot_internal_batch_tile(const drot_ctx* c, int key, int* rows, int* per_item) {
  if (key < 0 || key >= drot_ctx::kBatchKeys || c->batch_rows[key] <= 0) return false;
  *rows = c->batch_rows[key];
  *per_item = c->batch_per[key];
  return true;
}

void drot_internal_set_batch_tile(drot_ctx* c, int key, int rows, int per_item) {
  if (key < 0 || key >= drot_ctx::kBatchKeys) return;
  c->batch_rows[key] = rows;
  c->batch_per[key] = per_item;
}

int drot_internal_batch_chunks(const drot_ctx* c, int key) {
  return key >= 0 && key < 4 ? c->batch_chunks[key] : 0;
}

void drot_internal_set_batch_chunks(drot_ctx* c, int key, int chunks) {
  if (key >= 0 && key < 4) c->batch_chunks[key] = chunks;
}

// Make the context's workspace at least `bytes` large for a batched solve.
// The single-problem binding lives in the same workspace and is released.
int drot_internal_ctx_prepare(drot_ctx* c, void** ws, size_t bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  drop_graph(c);
  c->bound = false;
  if (bytes > c->ws_bytes) {
    if (c->ws) {
      (void)hipDeviceSynchronize();
      (void)hipFree(c->ws);
      c->ws = nullptr;
      c->ws_bytes = 0;
    }
    const size_t want = bytes + bytes / 4;
    if (hipMalloc(&c->ws, want) != hipSuccess) {
      (void)hipGetLastError();
      c->ws = nullptr;
      return fail(DROT_ENOMEM, "workspace allocation of %zu bytes failed", want);
    }
    c->ws_bytes = want;
  }
  *ws = c->ws;
  return DROT_OK;
}

extern "C" {

const char* drot_version(void) { return "drot-mi355x 0.1.0 (gfx950)"; }

const char* drot_strerror(int s) {
  switch (s) {
    case DROT_OK: return "ok: stopping test met";
    case DROT_MAXITER: return "max_iter reached before the stopping test";
    case DROT_EINVAL: return "invalid argument";
    case DROT_EMASS: return "marginals are negative or have unequal mass";
    case DROT_ENONFINITE: return "non-finite value in the inputs or the iteration";
    case DROT_ENOMEM: return "out of device memory";
    case DROT_EDEVICE: return "no usable GPU or HIP runtime error";
    case DROT_EUNSUPPORTED: return "unsupported combination";
    case DROT_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* drot_last_error(void) { return g_last_error.c_str(); }

int drot_ctx_create(drot_ctx** out, int device) {
  if (!out) return fail(DROT_EINVAL, "ctx output pointer is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(DROT_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count)
    return fail(DROT_EINVAL, "device %d out of range [0, %d)", device, count);
  HIP_TRY(hipSetDevice(device));
  drot_ctx* c = new drot_ctx();
  c->device = device;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->wall_rate = (double)khz * 1000.0;
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&c->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    drot_ctx_destroy(c);
    return fail(DROT_EDEVICE, "stream or pinned allocation failed");
  }
  memset(c->st_host, 0, sizeof(DevState));
  *out = c;
  return DROT_OK;
}

int drot_ctx_destroy(drot_ctx* c) {
  if (!c) return DROT_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  drop_graph(c);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return DROT_OK;
}

int drot_bind_cost(drot_ctx* c, int64_t m, int64_t n, int dtype, const drot_cost* cost,
                   const void* p, const void* q, const drot_params* prm, void* X, int64_t ldx,
                   const double* mu0, const double* nu0, void* stream) {
  int rc = validate(m, n, dtype, cost, p, q, prm, X, ldx, mu0, nu0);
  if (rc) return rc;
  if ((rc = check_ctx(c))) return rc;
  Geometry g;
  if ((rc = choose_geometry(dtype, m, n, cost, X, ldx, prm, &g))) return rc;
  size_t offs[12];
  if ((rc = ensure_workspace(c, m, n, g, offs))) return rc;
  hipStream_t s = (hipStream_t)stream;
  drop_graph(c);
  c->bound = false;
  c->finished = false;
  c->dtype = dtype;
  c->prm = *prm;
  c->args.m = m;
  c->args.n = n;
  c->args.ldx = ldx;
  c->args.cost = *cost;
  c->args.p = p;
  c->args.q = q;
  c->args.X = X;
  c->args.mu0 = mu0;
  c->args.nu0 = nu0;
  c->geo = g;
  c->skipc = (prm->flags & DROT_FLAG_SKIP_C) != 0;
  // A float32 problem that asks for compensated sums stays on sweep + aux:
  // the one-workgroup path's lane partials are plain sums in the problem type.
  c->small = cost->kind == DROT_COST_DENSE &&
             !(prm->flags & (DROT_FLAG_SKIP_C | DROT_FLAG_TIME_SWEEP)) &&
             !(dtype == DROT_F32 && (prm->flags & DROT_FLAG_COMPENSATED)) &&
             prm->tile_rows == 0 && prm->tile_chunks == 0 && prm->tile_unroll == 0 &&
             prm->tile_groups == 0 && prm->cache_mode == DROT_CACHE_AUTO &&
             small_fits(dtype, m, n);
  c->pend = !c->small && aux_workgroups(m, n) < kAuxSplitMin;
  c->enq = 0;
  c->sweep_ms = 0.0;
  c->sweep_n = 0;
  char* base = static_cast<char*>(c->ws);
  c->st = reinterpret_cast<DevState*>(base + offs[0]);
  c->trace = reinterpret_cast<double*>(base + offs[1]);

  SweepArgs& sa = c->sa;
  sa = SweepArgs{};
  sa.cost_kind = cost->kind;
  sa.dim = cost->dim;
  sa.xs = cost->xs;
  sa.xt = cost->xt;
  sa.C = cost->kind == DROT_COST_COORDS ? nullptr : cost->data;
  sa.X = X;
  sa.p = p;
  sa.q = q;
  sa.colpart = base + offs[2];
  sa.rowpart = base + offs[3];
  sa.tiles = reinterpret_cast<double*>(base + offs[4]);
  sa.a = reinterpret_cast<double*>(base + offs[5]);
  sa.b = reinterpret_cast<double*>(base + offs[6]);
  sa.phi64 = reinterpret_cast<double*>(base + offs[7]);
  sa.psi64 = reinterpret_cast<double*>(base + offs[8]);
  sa.phiT = base + offs[9];
  sa.psiT = base + offs[10];
  sa.blockpart = reinterpret_cast<double*>(base + offs[11]);
  c->bp[0] = sa.blockpart;
  c->bp[1] = sa.blockpart + (size_t)aux_workgroups(m, n) * kSlots;
  sa.mu0 = mu0;
  sa.nu0 = nu0;
  sa.st = c->st;
  sa.trace = c->trace;
  sa.trace_cap = kTraceCap;
  sa.wall_rate = c->wall_rate;
  sa.g = g.g;

  // Problem block of the device state.
  DevState* h = c->st_host;
  memset(h, 0, sizeof(DevState));
  h->rho = prm->rho;
  h->tol = prm->tol;
  h->max_iter = prm->max_iter;
  h->tol_mode = prm->tol_mode;
  h->m = m;
  h->n = n;
  h->cscale = cost->kind == DROT_COST_COORDS ? cost->scale : 0.0;
  HIP_TRY(hipMemcpyAsync(c->st, h, sizeof(DevState), hipMemcpyHostToDevice, s));
  if (cost->kind == DROT_COST_COORDS && !(cost->scale > 0)) HIP_TRY(launch_maxc(sa, s));
  HIP_TRY(launch_prep(sa, s));
  const int mode = prm->x0_mode == DROT_X0_GIVEN ? kInitX : kInitPQ;
  HIP_TRY(launch_sweep(dtype, mode, g.tile, sa, s));
  HIP_TRY(launch_aux(dtype, mode, sa, s));
  HIP_TRY(hipMemcpyAsync(h, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));

  if (h->init_bad > 0)
    return fail(DROT_ENONFINITE,
                "initialisation found %.0f non-finite entries in C, X_0, p, q or the warm "
                "start, or negative entries in X_0",
                h->init_bad);
  if (h->init_neg > 0)
    return fail(DROT_EMASS, "%.0f marginal entries are negative", h->init_neg);
  const double eps = dtype == DROT_F32 ? 1.1920929e-07 : 2.220446049250313e-16;
  const double sp = h->sum_p, sq = h->sum_q;
  if (!(sp > 0) || std::fabs(sp - sq) > 8.0 * eps * std::max(sp, sq))
    return fail(DROT_EMASS, "sum(p) = %.17g and sum(q) = %.17g differ (or are not positive)", sp, sq);
  c->bound = true;
  return DROT_OK;
}

int drot_bind(drot_ctx* c, int64_t m, int64_t n, int dtype, const void* C, int64_t ldc,
              const void* p, const void* q, const drot_params* prm, void* X, int64_t ldx,
              const double* mu0, const double* nu0, void* stream) {
  drot_cost cost{};
  cost.kind = DROT_COST_DENSE;
  cost.data = C;
  cost.ld = ldc;
  return drot_bind_cost(c, m, n, dtype, &cost, p, q, prm, X, ldx, mu0, nu0, stream);
}

}  // extern "C"

namespace {

// Enqueue `count` iterations with individual launches (timed in groups when
// DROT_FLAG_TIME_SWEEP is set).
int run_eager(drot_ctx* c, hipStream_t s, int64_t count) {
  const bool timed = (c->prm.flags & DROT_FLAG_TIME_SWEEP) != 0;
  const int G = group_size(c);
  int rc = DROT_OK;
  int64_t done = 0;
  while (done < count) {
    const int k = (int)std::min<int64_t>(G, count - done);
    if (timed && (rc = ensure_events(c, 2 * k))) return rc;
    const int64_t first = c->enq;
    for (int t = 0; t < k; ++t) {
      if ((rc = launch_iteration(c, s, timed ? c->ev[2 * t] : nullptr,
                                 timed ? c->ev[2 * t + 1] : nullptr, t, first)))
        return rc;
      ++c->enq;
    }
    if ((rc = launch_group_end(c, s, k, first))) return rc;
    if (timed) {
      HIP_TRY(hipStreamSynchronize(s));
      if ((rc = harvest_events(c, k))) return rc;
    }
    done += k;
  }
  return DROT_OK;
}

}  // namespace

extern "C" int drot_iterate(drot_ctx* c, int64_t iters, void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound (call drot_bind first)");
  if (iters < 0) return fail(DROT_EINVAL, "iters must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const bool timed = (c->prm.flags & DROT_FLAG_TIME_SWEEP) != 0;
  c->finished = false;
  if (c->small) {
    // Bounded launches; the kernel stops by itself at the stopping test.
    constexpr int64_t kChunk = 4096;
    while (iters > 0) {
      const int64_t k = std::min(iters, kChunk);
      HIP_TRY(launch_small(c->dtype, c->sa, k, s));
      c->enq += k;
      iters -= k;
    }
    return DROT_OK;
  }
  if (c->prm.flags & DROT_FLAG_NO_GRAPH) return run_eager(c, s, iters);
  if ((rc = ensure_graph(c))) return rc;
  const int G = group_size(c);
  int64_t done = 0;
  if (c->skipc && (c->enq & 1) && iters > 0) {  // realign to a C-reading iteration
    if ((rc = run_eager(c, s, 1))) return rc;
    done = 1;
  }
  while (iters - done >= G) {
    HIP_TRY(hipGraphLaunch(c->gexec, s));
    c->enq += G;
    if (timed) {
      HIP_TRY(hipStreamSynchronize(s));
      if ((rc = harvest_events(c, timed_count(G)))) return rc;
    }
    done += G;
  }
  return run_eager(c, s, iters - done);
}

// Tile autotuning: every candidate is bound (initialisation pass included),
// warmed up for one graph and timed over `iters` iterations of graph replays
// with hipEvents around the whole run; the fastest is bound again with the
// caller's parameters.
extern "C" int drot_tune(drot_ctx* c, int64_t iters, drot_params* best, double* us_per_iter,
                         void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound (call drot_bind first)");
  if (!best) return fail(DROT_EINVAL, "best is NULL");
  if (c->prm.x0_mode != DROT_X0_PQ)
    return fail(DROT_EUNSUPPORTED, "tuning overwrites X: bind with x0_mode = DROT_X0_PQ");
  if (iters < 0) return fail(DROT_EINVAL, "iters must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const auto A = c->args;
  const drot_params user = c->prm;
  if (c->small) {
    // The one-workgroup path has no tile variants: time it, bind again, and
    // return the caller's parameters.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(DROT_EDEVICE, "hipEventCreate failed");
    }
    drot_params t = user;
    t.tol = 0.0;
    t.max_iter = 2 * (iters > 0 ? iters : 256) + 1;
    float ms = 0.f;
    rc = drot_bind_cost(c, A.m, A.n, c->dtype, &A.cost, A.p, A.q, &t, A.X, A.ldx, A.mu0, A.nu0,
                        stream);
    const int64_t k = iters > 0 ? iters : 256;
    if (!rc) rc = drot_iterate(c, k, stream);
    if (!rc && (hipEventRecord(e0, s) != hipSuccess || drot_iterate(c, k, stream) != DROT_OK ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(DROT_EDEVICE, "timing the one-workgroup path failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = drot_bind_cost(c, A.m, A.n, c->dtype, &A.cost, A.p, A.q, &user, A.X, A.ldx, A.mu0,
                             A.nu0, stream)))
      return rc;
    *best = user;
    if (us_per_iter) *us_per_iter = ms * 1e3 / (double)k;
    return DROT_OK;
  }
  drot_params trial = user;
  trial.tol = 0.0;
  trial.flags &= ~(DROT_FLAG_NO_GRAPH | DROT_FLAG_TIME_SWEEP);
  trial.check_every = user.check_every > 0 ? user.check_every : 32;
  const int64_t G = trial.check_every + (c->skipc && (trial.check_every & 1) ? 1 : 0);
  if (iters == 0) iters = 4 * G;
  iters = (iters + G - 1) / G * G;
  trial.max_iter = G + iters + 1;
  static const int kRows[] = {8, 16, 32};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(DROT_EDEVICE, "hipEventCreate failed");
  }
  double best_ms = -1.0;
  drot_params winner = user;
  for (int rows : kRows)
    for (int chunks = 1; chunks <= 2 && !rc; ++chunks)
      for (int per = 1; per <= 2 && !rc; ++per) {
        const int64_t n_rb = (A.m + rows - 1) / rows;
        if (per == 2 && n_rb < 2) continue;
        drot_params t = trial;
        t.tile_rows = rows;
        t.tile_chunks = chunks;
        t.tile_groups = per == 1 ? 0 : (int)((n_rb + 1) / 2);
        rc = drot_bind_cost(c, A.m, A.n, c->dtype, &A.cost, A.p, A.q, &t, A.X, A.ldx, A.mu0,
                            A.nu0, stream);
        if (!rc) rc = drot_iterate(c, G, stream);
        if (rc) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(DROT_EDEVICE, "event record failed"); break; }
        if ((rc = drot_iterate(c, iters, stream))) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(DROT_EDEVICE, "event timing failed");
          break;
        }
        if (best_ms < 0 || ms < best_ms) {
          best_ms = ms;
          winner = user;
          winner.tile_rows = t.tile_rows;
          winner.tile_chunks = t.tile_chunks;
          winner.tile_groups = t.tile_groups;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = drot_bind_cost(c, A.m, A.n, c->dtype, &A.cost, A.p, A.q, &winner, A.X, A.ldx, A.mu0,
                           A.nu0, stream)))
    return rc;
  *best = winner;
  if (us_per_iter) *us_per_iter = best_ms * 1e3 / (double)iters;
  return DROT_OK;
}

extern "C" {

int drot_poll(drot_ctx* c, int64_t* iters_done, int32_t* stopped, void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters_done) *iters_done = c->st_host->iter;
  if (stopped) *stopped = c->st_host->done;
  return DROT_OK;
}

int drot_finish(drot_ctx* c, double* mu, double* nu, drot_result* out, void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound");
  if (!out) return fail(DROT_EINVAL, "out is NULL");
  hipStream_t s = (hipStream_t)stream;
  SweepArgs sa = c->sa;
  sa.mu_out = mu;
  sa.nu_out = nu;
  // Under the skip-C schedule an odd iteration count leaves W = X - rho C in
  // the array; the final pass then restores X while evaluating it.
  HIP_TRY(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int fmode = (c->skipc && (c->st_host->iter & 1)) ? kFinalW : kFinal;
  HIP_TRY(launch_sweep(c->dtype, fmode, c->geo.tile, sa, s));
  HIP_TRY(launch_aux(c->dtype, fmode, sa, s));
  HIP_TRY(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const DevState* h = c->st_host;
  memset(out, 0, sizeof(*out));
  out->iters = h->iter;
  out->status = h->done ? h->status : DROT_MAXITER;
  out->path = c->small ? 1 : 0;
  out->objective = h->f_pobj;
  out->dual_objective = h->f_dobj;
  out->r_primal = h->f_rp;
  out->r_dual = h->f_rd;
  out->gap = h->f_gap;
  out->eps_primal = h->f_eps_p;
  out->eps_dual = h->f_eps_d;
  out->eps_gap = h->f_eps_g;
  const uint64_t t1 = h->done ? h->t_stop : h->t_last;
  out->seconds_to_tol = (double)(t1 - h->t_start) / c->wall_rate;
  out->sweep_ms_total = c->sweep_ms;
  out->sweep_timed = c->sweep_n;
  out->cost_scale = c->sa.cost_kind == kCostCoords ? h->cscale : 0.0;
  c->finished = true;
  if (out->status == -3)
    return fail(DROT_ENONFINITE, "the iteration produced a non-finite value at iteration %lld",
                (long long)h->stop_iter);
  return out->status;
}

// Checkpoint layout (host memory): header, the device state record, the
// vectors a, b, phi (FP64), psi (FP64), phi, psi (element type), the trace.
struct CkptHeader {
  char magic[8];  // "DROTCKP1"
  int64_t m, n;
  int32_t dtype, cost_kind;
  int64_t enq;    // iterations enqueued since bind
  int32_t skipc, pad;
  uint64_t bytes; // total size
};

static size_t ckpt_bytes(const drot_ctx* c) {
  const int64_t m = c->args.m, n = c->args.n;
  const size_t es = c->dtype == DROT_F32 ? 4 : 8;
  return sizeof(CkptHeader) + sizeof(DevState) + sizeof(double) * (size_t)(2 * m + 2 * n) +
         es * (size_t)(m + n) + sizeof(double) * kTraceCap * kTraceWidth;
}

int drot_checkpoint_size(drot_ctx* c, size_t* bytes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound");
  if (!bytes) return fail(DROT_EINVAL, "bytes is NULL");
  *bytes = ckpt_bytes(c);
  return DROT_OK;
}

int drot_checkpoint(drot_ctx* c, void* host_buf, size_t bytes, void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound");
  if (!host_buf || bytes < ckpt_bytes(c))
    return fail(DROT_EINVAL, "checkpoint buffer of %zu bytes is too small (%zu needed)", bytes,
                ckpt_bytes(c));
  if (c->skipc && (c->enq & 1))
    return fail(DROT_ESTATE, "under the skip-C schedule X holds X - rho C after an odd number of "
                             "iterations: checkpoint after an even number");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t m = c->args.m, n = c->args.n;
  const size_t es = c->dtype == DROT_F32 ? 4 : 8;
  char* out = static_cast<char*>(host_buf);
  CkptHeader h{};
  memcpy(h.magic, "DROTCKP1", 8);
  h.m = m;
  h.n = n;
  h.dtype = c->dtype;
  h.cost_kind = c->args.cost.kind;
  h.enq = c->enq;
  h.skipc = c->skipc;
  h.bytes = ckpt_bytes(c);
  memcpy(out, &h, sizeof h);
  size_t o = sizeof h;
  const struct {
    const void* src;
    size_t len;
  } parts[] = {{c->st, sizeof(DevState)},       {c->sa.a, sizeof(double) * m},
               {c->sa.b, sizeof(double) * n},    {c->sa.phi64, sizeof(double) * m},
               {c->sa.psi64, sizeof(double) * n}, {c->sa.phiT, es * m},
               {c->sa.psiT, es * n},             {c->trace, sizeof(double) * kTraceCap * kTraceWidth}};
  for (const auto& part : parts) {
    HIP_TRY(hipMemcpy(out + o, part.src, part.len, hipMemcpyDeviceToHost));
    o += part.len;
  }
  return DROT_OK;
}

int drot_resume(drot_ctx* c, const void* host_buf, size_t bytes, void* stream) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "bind the problem (with X holding the checkpointed plan) first");
  if (!host_buf || bytes < sizeof(CkptHeader)) return fail(DROT_EINVAL, "checkpoint too small");
  CkptHeader h;
  memcpy(&h, host_buf, sizeof h);
  if (memcmp(h.magic, "DROTCKP1", 8) != 0) return fail(DROT_EINVAL, "not a DROT checkpoint");
  if (h.m != c->args.m || h.n != c->args.n || h.dtype != c->dtype ||
      h.cost_kind != c->args.cost.kind || (h.skipc != 0) != c->skipc)
    return fail(DROT_EINVAL, "checkpoint of a %lldx%lld problem (dtype %d, cost %d, skip-C %d) "
                             "does not match the bound problem",
                (long long)h.m, (long long)h.n, h.dtype, h.cost_kind, h.skipc);
  if (h.bytes != ckpt_bytes(c) || bytes < h.bytes) return fail(DROT_EINVAL, "checkpoint size mismatch");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t m = c->args.m, n = c->args.n;
  const size_t es = c->dtype == DROT_F32 ? 4 : 8;
  const char* in = static_cast<const char*>(host_buf);
  size_t o = sizeof h;
  const struct {
    void* dst;
    size_t len;
  } parts[] = {{c->st, sizeof(DevState)},       {c->sa.a, sizeof(double) * m},
               {c->sa.b, sizeof(double) * n},    {c->sa.phi64, sizeof(double) * m},
               {c->sa.psi64, sizeof(double) * n}, {c->sa.phiT, es * m},
               {c->sa.psiT, es * n},             {c->trace, sizeof(double) * kTraceCap * kTraceWidth}};
  for (const auto& part : parts) {
    HIP_TRY(hipMemcpy(part.dst, in + o, part.len, hipMemcpyHostToDevice));
    o += part.len;
  }
  // The bound run's tolerances and limits apply from here on.
  DevState* st = c->st_host;
  memcpy(st, in + sizeof h, sizeof(DevState));
  st->tol = c->prm.tol;
  st->max_iter = c->prm.max_iter;
  st->tol_mode = c->prm.tol_mode;
  st->done = 0;
  st->status = 0;
  HIP_TRY(hipMemcpy(c->st, st, sizeof(DevState), hipMemcpyHostToDevice));
  // Fresh time origin and completion counter (the prep kernel; without a warm
  // start its sums of phi_0 and psi_0 are zero and no longer used).
  SweepArgs sa = c->sa;
  sa.mu0 = nullptr;
  sa.nu0 = nullptr;
  HIP_TRY(launch_prep(sa, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->enq = h.enq;
  c->finished = false;
  return DROT_OK;
}

int drot_get_trace(drot_ctx* c, int64_t first, int64_t count, double* host_out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->bound) return fail(DROT_ESTATE, "no problem bound");
  if (!host_out || count < 0) return fail(DROT_EINVAL, "bad output buffer or count");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
  const int64_t last = c->st_host->iter;
  if (first < 1 || first + count - 1 > last || last - first >= kTraceCap)
    return fail(DROT_EINVAL, "records [%lld, %lld] not available (have up to %lld, keep %d)",
                (long long)first, (long long)(first + count - 1), (long long)last, kTraceCap);
  for (int64_t k = first; k < first + count; ++k) {
    const int64_t slot = (k - 1) % kTraceCap;
    HIP_TRY(hipMemcpy(host_out + (k - first) * kTraceWidth, c->trace + slot * kTraceWidth,
                      sizeof(double) * kTraceWidth, hipMemcpyDeviceToHost));
  }
  return DROT_OK;
}

int drot_solve_cost(drot_ctx* c, int64_t m, int64_t n, int dtype, const drot_cost* cost,
                    const void* p, const void* q, const drot_params* prm, void* X, int64_t ldx,
                    double* mu, double* nu, const double* mu0, const double* nu0,
                    drot_result* out, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!out) return fail(DROT_EINVAL, "out is NULL");
  int rc = validate(m, n, dtype, cost, p, q, prm, X, ldx, mu0, nu0);
  if (rc) return rc;
  if ((rc = drot_bind_cost(c, m, n, dtype, cost, p, q, prm, X, ldx, mu0, nu0, stream))) return rc;
  const int G = group_size(c);
  int64_t done_iters = 0;
  int32_t stopped = 0;
  while (!stopped && done_iters < prm->max_iter) {
    const int64_t k = std::min<int64_t>(G, prm->max_iter - done_iters);
    if ((rc = drot_iterate(c, k, stream))) return rc;
    if ((rc = drot_poll(c, &done_iters, &stopped, stream))) return rc;
  }
  rc = drot_finish(c, mu, nu, out, stream);
  out->seconds_total =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int drot_solve(drot_ctx* c, int64_t m, int64_t n, int dtype, const void* C, int64_t ldc,
               const void* p, const void* q, const drot_params* prm, void* X, int64_t ldx,
               double* mu, double* nu, const double* mu0, const double* nu0, drot_result* out,
               void* stream) {
  drot_cost cost{};
  cost.kind = DROT_COST_DENSE;
  cost.data = C;
  cost.ld = ldc;
  return drot_solve_cost(c, m, n, dtype, &cost, p, q, prm, X, ldx, mu, nu, mu0, nu0, out, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// drot_solve without allocation: the workspace is a static device array.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

// Device-side workspace of drot_solve_noalloc, one copy per GPU for the life
// of the process.  In host code `scratch` names a host-side stand-in: its
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices)
    return fail(DROT_EDEVICE, "device %d beyond the %d the static scratch supports", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DROT_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return DROT_OK;
}

}  // namespace

extern "C" int drot_solve_noalloc(int64_t m, int64_t n, int dtype, const void* C, int64_t ldc,
                                  const void* p, const void* q, const drot_params* params,
                                  void* X, int64_t ldx, double* mu, double* nu, const double* mu0,
                                  const double* nu0, drot_result* out, void* stream) {
  if (!out) return fail(DROT_EINVAL, "out is NULL");
  drot_cost cost{};
  cost.kind = DROT_COST_DENSE;
  cost.data = C;
  cost.ld = ldc;
  int rc = validate(m, n, dtype, &cost, p, q, params, X, ldx, mu0, nu0);
  if (rc) return rc;
  if (params->flags & DROT_FLAG_TIME_SWEEP)
    return fail(DROT_EUNSUPPORTED, "sweep timing needs events, which drot_solve_noalloc does not "
                                   "create");
  // Size check before any device call.
  Geometry g;
  if ((rc = choose_geometry(dtype, m, n, &cost, X, ldx, params, &g))) return rc;
  size_t offs[12];
  const size_t need = workspace_layout(m, n, g, offs);
  if (need > kScratchBytes)
    return fail(DROT_EINVAL,
                "a %lld x %lld problem needs %zu bytes of workspace, more than the %zu bytes of "
                "static scratch of drot_solve_noalloc",
                (long long)m, (long long)n, need, kScratchBytes);
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  void* ptr = nullptr;
  if ((rc = scratch_address(device, &ptr))) return rc;

  drot_ctx c;  // on the stack: no stream, no pinned memory, no graphs, no events
  c.device = device;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c.wall_rate = (double)khz * 1000.0;
  DevState host_state{};
  c.st_host = &host_state;
  c.ws = ptr;
  c.ws_bytes = kScratchBytes;
  c.fixed_ws = true;
  drot_params prm = *params;
  prm.flags |= DROT_FLAG_NO_GRAPH;  // launches only: instantiating a graph allocates
  return drot_solve_cost(&c, m, n, dtype, &cost, p, q, &prm, X, ldx, mu, nu, mu0, nu0, out,
                         stream);
}
